// Device building blocks shared by the single-graph and batched solvers: a
// 128 x 128 register-blocked min-plus tile update (arXiv:1902.04446, Table 1
// MinPlus = MatProd then MatMin) and the Floyd-Warshall closure of a
// diagonal block held in the same register layout (Table 1 FloydWarshall).
//
// Register layout of a 128 x 128 tile over 256 threads: thread (tx, ty) =
// (t % 16, t / 16) holds acc[m][e] = C[row(m)][col(e)] with
// row(m) = (m / 4) * 64 + ty * 4 + m % 4 and col(e) = (e / 4) * 64 + tx * 4 + e % 4.
#pragma once

#include "apsp_common.h"

namespace apsp {
namespace tile {

constexpr int TB = kRoundB;  // tile edge == round width
constexpr int KC = 16;       // k values per LDS stage
constexpr int NT = 256;      // threads per tile workgroup

// LDS of one tile workgroup: two stages of the column-panel operand, stored
// as k-pairs (a[i][k], a[i][k+1]), and of the row-panel operand.
struct Lds {
    uint2 As[2][KC / 2][TB];
    uint4 Bs[2][KC][TB / 4];
};

__device__ __forceinline__ uint4 ld4(const uint32_t *p) {
    return *reinterpret_cast<const uint4 *>(p);
}
__device__ __forceinline__ void st4(uint32_t *p, uint4 v) { *reinterpret_cast<uint4 *>(p) = v; }

// Non-temporal 16-byte load/store (nt bit): for output tiles that are read
// and written once per pass, so they do not evict panel blocks other
// workgroups still read from L2.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ uint4 ld4_stream(const uint32_t *p) {
    const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4_stream(uint32_t *p, uint4 v) {
    const u32x4 w = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(w, reinterpret_cast<u32x4 *>(p));
}

// Wave priority of the launches on the rounds' critical chain (phase 1,
// phase 2, the tiles the next round's phases read first, the deferred
// updates).  They share CUs with the bulk phase-3 launches, whose waves are
// older and almost always ready to issue; at equal priority the chain's waves
// (a 128-pivot closure with a barrier per pivot above all) then wait for
// issue slots and the next round's phases start late.
__device__ __forceinline__ void chain_priority() { __builtin_amdgcn_s_setprio(3); }

__device__ __forceinline__ int row_of(int m, int ty) { return (m >> 2) * 64 + ty * 4 + (m & 3); }
__device__ __forceinline__ int col_of(int e, int tx) { return (e >> 2) * 64 + tx * 4 + (e & 3); }

// Load the mr x nc tile at (i0, j0) into acc; entries outside are padded with
// "no edge".  NORM applies the input normalisation on the way in (Op::norm:
// int32 values above 2^30 -> 2^30, or the conversion of OpI32F; a tile on the
// diagonal gets a zero diagonal).  store_acc converts back with Op::out.
// STREAM: non-temporal loads (see ld4_stream).
template <class Op, bool NORM, bool STREAM = false>
__device__ __forceinline__ void load_acc(uint32_t (&acc)[8][8], const uint32_t *D, int64_t ld,
                                         int64_t i0, int64_t j0, int mr, int nc, bool vec) {
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const uint32_t PAD = Op::pad();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int row = row_of(m, ty);
        const uint32_t *crow = D + (i0 + (row < mr ? row : mr - 1)) * ld + j0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int col = h * 64 + tx * 4;
            if (vec && row < mr && col + 3 < nc) {
                const uint4 c4 = STREAM ? ld4_stream(crow + col) : ld4(crow + col);
                acc[m][h * 4 + 0] = c4.x;
                acc[m][h * 4 + 1] = c4.y;
                acc[m][h * 4 + 2] = c4.z;
                acc[m][h * 4 + 3] = c4.w;
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const uint32_t x = crow[col + e < nc ? col + e : nc - 1];
                    acc[m][h * 4 + e] = (row < mr && col + e < nc) ? x : PAD;
                }
            }
        }
    }
    if (NORM) {
#pragma unroll
        for (int m = 0; m < 8; ++m)
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[m][e] = Op::norm(acc[m][e]);
        if (i0 == j0) {
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (row_of(m, ty) == col_of(e, tx)) acc[m][e] = 0u;
        }
    }
}

template <class Op, bool STREAM = false>
__device__ __forceinline__ void store_acc(const uint32_t (&acc)[8][8], uint32_t *D, int64_t ld,
                                          int64_t i0, int64_t j0, int mr, int nc, bool vec) {
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int row = row_of(m, ty);
        if (row >= mr) continue;
        uint32_t *crow = D + (i0 + row) * ld + j0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int col = h * 64 + tx * 4;
            if (vec && col + 3 < nc) {
                const uint4 o4 = make_uint4(Op::out(acc[m][h * 4 + 0]), Op::out(acc[m][h * 4 + 1]),
                                            Op::out(acc[m][h * 4 + 2]), Op::out(acc[m][h * 4 + 3]));
                if (STREAM)
                    st4_stream(crow + col, o4);
                else
                    st4(crow + col, o4);
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (col + e < nc) crow[col + e] = Op::out(acc[m][h * 4 + e]);
            }
        }
    }
}

// acc = min(acc, A (x) B) for the output tile of rows i0 .. i0+mr and
// columns j0 .. j0+nc, with A[i][k] = A[(i0 + i) * lda + k] and
// B[k][j] = B[k * ldb + j0 + j], k in [0, kw) (any kw >= 1).  k runs in
// stages of 16 through double-buffered LDS, prefetched into registers one
// stage ahead; one barrier per stage; every thread returns after a final
// barrier, so the LDS may be reused at once.  One min3 folds the two
// candidates of a k-pair:
//     c = min3(c, a[i][k] + b[k][j], a[i][k+1] + b[k+1][j])
// (2 adds + 1 min3 per 2 updates).  Out-of-range rows, columns and k read
// as "no edge", which never wins a minimum.  The operands are read from
// global memory only, so C may be one of them as long as it is stored after
// this returns (phase 2).  `vec` promises 16-byte aligned rows of A and B.
//
// TA / TB read an operand from its transpose (symmetric storage):
//   TA: A[i][k] = A[k * lda + i0 + i]      TB: B[k][j] = B[(j0 + j) * ldb + k]
// The transposed loaders read rows of the stored matrix (coalesced) and
// scatter them into the same LDS layout.
// PARTIAL: a tile whose valid rows (mr <= 64) or columns (nc <= 64) fit in
// the first half updates only those (acc rows m < 4 / columns e < 4, by
// quadrant, on workgroup-uniform branches); the other accumulators keep
// their values.
template <class Op, bool NORM, bool TA = false, bool TB = false, bool PARTIAL = false>
__device__ __forceinline__ void minplus_tile_ab(uint32_t (&acc)[8][8], const uint32_t *A, int64_t lda,
                                                const uint32_t *B, int64_t ldb, int64_t i0,
                                                int64_t j0, int mr, int nc, int kw, bool vec,
                                                Lds &L) {
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const uint32_t PAD = Op::pad();
    // direct A: row ar, k offset ak..ak+7 of a stage; transposed A: stored
    // row (k) t/16 of a stage, columns (i) (t%16)*8 .. +7
    const int ar = TA ? (t >> 4) : (t >> 1), ak = TA ? (t & 15) * 8 : (t & 1) * 8;
    // direct B: k row br of a stage, columns bc..bc+7; transposed B: stored
    // row (j) t/2, columns (k) (t%2)*8 .. +7 of a stage
    const int br = TB ? (t >> 1) : (t >> 4), bc = TB ? (t & 1) * 8 : (t & 15) * 8;
    const uint32_t *Arow = TA ? (A + i0) : (A + (i0 + (ar < mr ? ar : mr - 1)) * lda);
    const uint32_t *Bbase = TB ? (B + (j0 + (br < nc ? br : nc - 1)) * ldb) : (B + j0);
    const int64_t ld = ldb;

    uint32_t pa[8], pb[8];
    auto gload_t = [&](int c) {
        if (TA) {  // 8 values of stored row k = c*KC + ar: A[ak .. ak+7][k]
            const int kr = c * KC + ar;
            const uint32_t *row = Arow + (int64_t)(kr < kw ? kr : kw - 1) * lda;
            if (vec && kr < kw && ak + 8 <= mr) {
                const uint4 x0 = ld4(row + ak), x1 = ld4(row + ak + 4);
                pa[0] = x0.x; pa[1] = x0.y; pa[2] = x0.z; pa[3] = x0.w;
                pa[4] = x1.x; pa[5] = x1.y; pa[6] = x1.z; pa[7] = x1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t x = row[ak + e < mr ? ak + e : mr - 1];
                    pa[e] = (kr < kw && ak + e < mr) ? x : PAD;
                }
            }
        }
        if (TB) {  // 8 values of stored row j = br: B[c*KC + bc .. +7][j]
            const int kk = c * KC + bc;
            if (vec && br < nc && kk + 8 <= kw) {
                const uint4 y0 = ld4(Bbase + kk), y1 = ld4(Bbase + kk + 4);
                pb[0] = y0.x; pb[1] = y0.y; pb[2] = y0.z; pb[3] = y0.w;
                pb[4] = y1.x; pb[5] = y1.y; pb[6] = y1.z; pb[7] = y1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t x = Bbase[kk + e < kw ? kk + e : kw - 1];
                    pb[e] = (br < nc && kk + e < kw) ? x : PAD;
                }
            }
        }
    };
    auto gload = [&](int c) {
        gload_t(c);
        if (!TA) {
            const int kk = c * KC + ak;
            if (vec && ar < mr && kk + 8 <= kw) {
                const uint4 x0 = ld4(Arow + kk), x1 = ld4(Arow + kk + 4);
                pa[0] = x0.x; pa[1] = x0.y; pa[2] = x0.z; pa[3] = x0.w;
                pa[4] = x1.x; pa[5] = x1.y; pa[6] = x1.z; pa[7] = x1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t x = Arow[kk + e < kw ? kk + e : kw - 1];
                    pa[e] = (ar < mr && kk + e < kw) ? x : PAD;
                }
            }
        }
        if (!TB) {
            const int kr = c * KC + br;
            const uint32_t *brow = Bbase + (int64_t)(kr < kw ? kr : kw - 1) * ld;
            if (vec && kr < kw && bc + 8 <= nc) {
                const uint4 y0 = ld4(brow + bc), y1 = ld4(brow + bc + 4);
                pb[0] = y0.x; pb[1] = y0.y; pb[2] = y0.z; pb[3] = y0.w;
                pb[4] = y1.x; pb[5] = y1.y; pb[6] = y1.z; pb[7] = y1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const uint32_t x = brow[bc + e < nc ? bc + e : nc - 1];
                    pb[e] = (kr < kw && bc + e < nc) ? x : PAD;
                }
            }
        }
        if (NORM) {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                pa[e] = Op::norm(pa[e]);
                pb[e] = Op::norm(pb[e]);
            }
        }
    };
    auto sstore = [&](int s) {
        if (TA) {  // element (k = ar, i = ak + e) -> word (k/2, i, k%2) of As
            uint32_t *w = reinterpret_cast<uint32_t *>(&L.As[s][ar >> 1][0]) + (ar & 1);
#pragma unroll
            for (int e = 0; e < 8; ++e) w[2 * (ak + e)] = pa[e];
        } else {
#pragma unroll
            for (int p = 0; p < 4; ++p)
                L.As[s][(ak >> 1) + p][ar] = make_uint2(pa[2 * p], pa[2 * p + 1]);
        }
        if (TB) {  // element (k = bc + e, j = br) -> word j of row k of Bs
#pragma unroll
            for (int e = 0; e < 8; ++e)
                reinterpret_cast<uint32_t *>(&L.Bs[s][bc + e][0])[br] = pb[e];
        } else {
            L.Bs[s][br][(bc >> 2) + 0] = make_uint4(pb[0], pb[1], pb[2], pb[3]);
            L.Bs[s][br][(bc >> 2) + 1] = make_uint4(pb[4], pb[5], pb[6], pb[7]);
        }
    };

    const int nch = (kw + KC - 1) / KC;
    gload(0);
    sstore(0);
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int s = c & 1;
        if (c + 1 < nch) gload(c + 1);
#pragma unroll 2
        for (int p = 0; p < KC / 2; ++p) {
            uint32_t a0[8], a1[8], b0[8], b1[8];
            if (!PARTIAL) {
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const uint2 av = L.As[s][p][row_of(m, ty)];
                    a0[m] = av.x;
                    a1[m] = av.y;
                }
                const uint4 b00 = L.Bs[s][2 * p][tx], b01 = L.Bs[s][2 * p][16 + tx];
                const uint4 b10 = L.Bs[s][2 * p + 1][tx], b11 = L.Bs[s][2 * p + 1][16 + tx];
                b0[0] = b00.x; b0[1] = b00.y; b0[2] = b00.z; b0[3] = b00.w;
                b0[4] = b01.x; b0[5] = b01.y; b0[6] = b01.z; b0[7] = b01.w;
                b1[0] = b10.x; b1[1] = b10.y; b1[2] = b10.z; b1[3] = b10.w;
                b1[4] = b11.x; b1[5] = b11.y; b1[6] = b11.z; b1[7] = b11.w;
#pragma unroll
                for (int m = 0; m < 8; ++m)
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        acc[m][e] = Op::min3(acc[m][e], Op::add(a0[m], b0[e]), Op::add(a1[m], b1[e]));
            } else {
                const bool rows2 = mr > 64, cols2 = nc > 64;  // uniform
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const uint2 av = L.As[s][p][row_of(m, ty)];
                    a0[m] = av.x;
                    a1[m] = av.y;
                }
                const uint4 b00 = L.Bs[s][2 * p][tx], b10 = L.Bs[s][2 * p + 1][tx];
                b0[0] = b00.x; b0[1] = b00.y; b0[2] = b00.z; b0[3] = b00.w;
                b1[0] = b10.x; b1[1] = b10.y; b1[2] = b10.z; b1[3] = b10.w;
#pragma unroll
                for (int m = 0; m < 4; ++m)
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        acc[m][e] = Op::min3(acc[m][e], Op::add(a0[m], b0[e]), Op::add(a1[m], b1[e]));
                if (cols2) {
                    const uint4 b01 = L.Bs[s][2 * p][16 + tx], b11 = L.Bs[s][2 * p + 1][16 + tx];
                    b0[4] = b01.x; b0[5] = b01.y; b0[6] = b01.z; b0[7] = b01.w;
                    b1[4] = b11.x; b1[5] = b11.y; b1[6] = b11.z; b1[7] = b11.w;
#pragma unroll
                    for (int m = 0; m < 4; ++m)
#pragma unroll
                        for (int e = 4; e < 8; ++e)
                            acc[m][e] = Op::min3(acc[m][e], Op::add(a0[m], b0[e]), Op::add(a1[m], b1[e]));
                }
                if (rows2) {
#pragma unroll
                    for (int m = 4; m < 8; ++m) {
                        const uint2 av = L.As[s][p][row_of(m, ty)];
                        a0[m] = av.x;
                        a1[m] = av.y;
                    }
#pragma unroll
                    for (int m = 4; m < 8; ++m)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[m][e] = Op::min3(acc[m][e], Op::add(a0[m], b0[e]), Op::add(a1[m], b1[e]));
                    if (cols2) {
#pragma unroll
                        for (int m = 4; m < 8; ++m)
#pragma unroll
                            for (int e = 4; e < 8; ++e)
                                acc[m][e] = Op::min3(acc[m][e], Op::add(a0[m], b0[e]),
                                                     Op::add(a1[m], b1[e]));
                    }
                }
            }
        }
        if (c + 1 < nch) sstore(s ^ 1);
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Direct staging for full 128 x 128 tiles.  Both operands are copied from
// global memory into LDS by the load unit itself (global_load_lds_dwordx4:
// each lane's 16 bytes land at LDS base + 16 * lane), with no register
// round trip, so a workgroup holds 117 VGPRs per thread instead of ~140 and a
// CU runs 4 workgroups instead of 3.  That needs both operands k-major in
// memory: B is (row panel rows are k), A is supplied transposed,
// AT[k][i] = A[i][k] (a transposed copy of the column panel).  LDS per stage:
// A[k][i] and B[k][j], 16 k rows of 128 values each, as 16-byte chunks.
// ---------------------------------------------------------------------------
struct LdsDirect {
    uint4 A[2][KC][TB / 4];
    uint4 B[2][KC][TB / 4];
};
static_assert(sizeof(LdsDirect) == sizeof(Lds), "direct staging reuses the tile LDS");

typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ void dma16(const uint32_t *g, uint4 *l) {
    __builtin_amdgcn_global_load_lds(g, (lds_void_t *)l, 16, 0, 0);
}

// acc = min(acc, A (x) B) for a full 128 x 128 output tile at (i0, j0), k in
// [0, kw), kw a multiple of 16, with A[i][k] = AT[k][i] taken from AT0 for
// k < ksplit and from AT1 (row k - ksplit) otherwise (ksplit a multiple of 16;
// the two column panels of a round pair), both with leading dimension ldat,
// and B[k][j] = B[k * ldb + j0 + j].  Every row read is 16-byte aligned and
// in bounds (the caller guarantees full tiles).  One barrier per stage; the
// stage after next is loaded while a stage is computed; every thread returns
// after a final barrier.  Same candidates and minima as minplus_tile_ab, so
// the same bits.
template <class Op>
__device__ __forceinline__ void minplus_tile_direct(uint32_t (&acc)[8][8], const uint32_t *AT0,
                                                    const uint32_t *AT1, int ksplit, int64_t ldat,
                                                    const uint32_t *B, int64_t ldb, int64_t i0,
                                                    int64_t j0, int kw, Lds &Lraw) {
    LdsDirect &L = reinterpret_cast<LdsDirect &>(Lraw);
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);  // wave: LDS base must be uniform
    const int l = t & 63;
    // a wave's two loads per operand and stage: chunks p = 128 w + 64 h + l,
    // chunk p = (k row p / 32, 16-byte column chunk p % 32)
    // (32-bit element offsets from uniform bases: the caller keeps 16 ld + i0,
    // 16 ld + j0 below 2^30)
    const int p0 = 128 * w + l, p1 = p0 + 64;
    const uint32_t a_off0 = (uint32_t)(p0 >> 5) * (uint32_t)ldat + (uint32_t)i0 + (p0 & 31) * 4;
    const uint32_t a_off1 = a_off0 + 2u * (uint32_t)ldat;
    const uint32_t b_off0 = (uint32_t)(p0 >> 5) * (uint32_t)ldb + (uint32_t)j0 + (p0 & 31) * 4;
    const uint32_t b_off1 = b_off0 + 2u * (uint32_t)ldb;
    auto issue = [&](int c, int s) {
        const int k0 = c * KC;
        const uint32_t *ab = k0 < ksplit ? AT0 + (int64_t)k0 * ldat : AT1 + (int64_t)(k0 - ksplit) * ldat;
        const uint32_t *bb = B + (int64_t)k0 * ldb;
        uint4 *la = &L.A[s][0][0] + 128 * w;
        uint4 *lb = &L.B[s][0][0] + 128 * w;
        dma16(ab + a_off0, la);
        dma16(ab + a_off1, la + 64);
        dma16(bb + b_off0, lb);
        dma16(bb + b_off1, lb + 64);
    };
    const int nch = kw / KC;
    issue(0, 0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    for (int c = 0; c < nch; ++c) {
        const int s = c & 1;
        // buffer s^1 was last read in stage c-1, which every wave has left
        if (c + 1 < nch) issue(c + 1, s ^ 1);
#pragma unroll 2
        for (int p = 0; p < KC / 2; ++p) {
            uint32_t a0[8], a1[8], b0[8], b1[8];
            // rows row_of(m, ty): ty*4 .. +3 (m < 4) and 64 + ty*4 .. +3
            const uint4 x00 = L.A[s][2 * p][ty], x01 = L.A[s][2 * p][16 + ty];
            const uint4 x10 = L.A[s][2 * p + 1][ty], x11 = L.A[s][2 * p + 1][16 + ty];
            a0[0] = x00.x; a0[1] = x00.y; a0[2] = x00.z; a0[3] = x00.w;
            a0[4] = x01.x; a0[5] = x01.y; a0[6] = x01.z; a0[7] = x01.w;
            a1[0] = x10.x; a1[1] = x10.y; a1[2] = x10.z; a1[3] = x10.w;
            a1[4] = x11.x; a1[5] = x11.y; a1[6] = x11.z; a1[7] = x11.w;
            const uint4 b00 = L.B[s][2 * p][tx], b01 = L.B[s][2 * p][16 + tx];
            const uint4 b10 = L.B[s][2 * p + 1][tx], b11 = L.B[s][2 * p + 1][16 + tx];
            b0[0] = b00.x; b0[1] = b00.y; b0[2] = b00.z; b0[3] = b00.w;
            b0[4] = b01.x; b0[5] = b01.y; b0[6] = b01.z; b0[7] = b01.w;
            b1[0] = b10.x; b1[1] = b10.y; b1[2] = b10.z; b1[3] = b10.w;
            b1[4] = b11.x; b1[5] = b11.y; b1[6] = b11.z; b1[7] = b11.w;
#pragma unroll
            for (int m = 0; m < 8; ++m)
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    acc[m][e] = Op::min3(acc[m][e], Op::add(a0[m], b0[e]), Op::add(a1[m], b1[e]));
        }
        // the next stage's operands are in LDS and every wave is done with this one
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();
    }
}

// Load (store == false) or store a full 128 x 128 tile at `base` (leading
// dimension ld, 16-byte aligned rows), in the accumulator layout, with no
// conversion (the Ops whose memory form is their compute form: OpF32,
// OpI32).  The tile is addressed as one uniform base pointer plus 32-bit lane
// offsets (the caller guarantees 128 ld < 2^30); a caller that forms base and
// ld again for the store behind an empty asm statement keeps no 64-bit row
// address live across the products, which saves the registers of a
// workgroup at 4 per CU.
__device__ __forceinline__ void io_direct(uint32_t (&acc)[8][8], uint32_t *base, uint32_t ld,
                                          bool store) {
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const uint32_t off = (uint32_t)row_of(m, ty) * ld + (uint32_t)tx * 4u;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint32_t *p = base + off + h * 64;
            if (store) {
                st4_stream(p, make_uint4(acc[m][h * 4 + 0], acc[m][h * 4 + 1], acc[m][h * 4 + 2],
                                         acc[m][h * 4 + 3]));
            } else {
                const uint4 v = ld4_stream(p);
                acc[m][h * 4 + 0] = v.x;
                acc[m][h * 4 + 1] = v.y;
                acc[m][h * 4 + 2] = v.z;
                acc[m][h * 4 + 3] = v.w;
            }
        }
    }
}

// Store the mr x nc tile transposed: dst[col * ldd + i0 + row] = C[row][col]
// (Op::out applied), the layout minplus_tile_direct takes its A operand in.
// dst and ldd must keep 16-byte alignment at i0 (i0 a multiple of 4).
template <class Op>
__device__ __forceinline__ void store_acc_t(const uint32_t (&acc)[8][8], uint32_t *dst, int64_t ldd,
                                            int64_t i0, int mr, int nc) {
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int col = col_of(e, tx);
        if (col >= nc) continue;
        uint32_t *drow = dst + (int64_t)col * ldd + i0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = h * 64 + ty * 4;
            if (row + 3 < mr) {
                st4(drow + row, make_uint4(Op::out(acc[h * 4 + 0][e]), Op::out(acc[h * 4 + 1][e]),
                                           Op::out(acc[h * 4 + 2][e]), Op::out(acc[h * 4 + 3][e])));
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (row + u < mr) drow[row + u] = Op::out(acc[h * 4 + u][e]);
            }
        }
    }
}

// The blocked method's form: A = D[i0.., kb .. kb+kw), B = D[kb .. kb+kw, j0..].
template <class Op, bool NORM, bool PARTIAL = false>
__device__ __forceinline__ void minplus_tile(uint32_t (&acc)[8][8], const uint32_t *D, int64_t ld,
                                             int64_t i0, int64_t j0, int64_t kb, int mr, int nc,
                                             int kw, bool vec, Lds &L) {
    minplus_tile_ab<Op, NORM, false, false, PARTIAL>(acc, D + kb, ld, D + kb * ld, ld, i0, j0, mr,
                                                     nc, kw, vec, L);
}

// ---------------------------------------------------------------------------
// Floyd-Warshall closure of a (kw x kw, kw <= 128) diagonal block held in
// registers in the layout above (thread (tx, ty) holds rows
// {ty*4 + m, 64 + ty*4 + m}, columns {tx*4 + e, 64 + tx*4 + e}).  Pivot k:
// the 16 threads holding row k and the 16 holding column k publish them to
// LDS (double-buffered, one barrier per pivot), then every thread applies
// d_ij = min(d_ij, d_ik + d_kj) to its entries.  Same operations in the same
// order as the textbook loop, so the same bits.  A block of kw <= 64
// vertices lives in acc rows m < 4, columns e < 4, and only that quadrant is
// updated.  `lds` needs 4 x 128 words; every thread returns after the last
// pivot's barrier.
//
// (Applying pivots in pairs, one barrier per pair and one min3 per entry,
// does fewer instructions but lengthens each barrier-to-barrier step; it
// measured slower on the rounds' critical chain.)
// ---------------------------------------------------------------------------
template <class Op>
__device__ __forceinline__ void close_block(uint32_t (&acc)[8][8], int kw, uint32_t *lds) {
    const int t = threadIdx.x, tx = t & 15, ty = t >> 4;
    const bool big = kw > 64;
    uint32_t *rowbuf = lds;            // [2][128]
    uint32_t *colbuf = lds + 2 * TB;   // [2][128]
    // pivots in ascending order: k = kh*64 + kq*4 + u
#pragma unroll
    for (int kh = 0; kh < 2; ++kh) {
        for (int kq = 0; kq < 16; ++kq) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = kh * 64 + kq * 4 + u;
                if (k < kw) {
                    const int sel = (k & 1) * TB;
                    const int mk = kh * 4 + u;  // register row/column index of pivot k
                    if (ty == kq) {
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            *reinterpret_cast<uint4 *>(&rowbuf[sel + h * 64 + tx * 4]) =
                                make_uint4(acc[mk][h * 4 + 0], acc[mk][h * 4 + 1],
                                           acc[mk][h * 4 + 2], acc[mk][h * 4 + 3]);
                    }
                    if (tx == kq) {
#pragma unroll
                        for (int h = 0; h < 2; ++h)
                            *reinterpret_cast<uint4 *>(&colbuf[sel + h * 64 + ty * 4]) =
                                make_uint4(acc[h * 4 + 0][mk], acc[h * 4 + 1][mk],
                                           acc[h * 4 + 2][mk], acc[h * 4 + 3][mk]);
                    }
                    __syncthreads();
                    uint32_t dik[8], dkj[8];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const uint4 c4 = *reinterpret_cast<const uint4 *>(&colbuf[sel + h * 64 + ty * 4]);
                        const uint4 r4 = *reinterpret_cast<const uint4 *>(&rowbuf[sel + h * 64 + tx * 4]);
                        dik[h * 4 + 0] = c4.x; dik[h * 4 + 1] = c4.y;
                        dik[h * 4 + 2] = c4.z; dik[h * 4 + 3] = c4.w;
                        dkj[h * 4 + 0] = r4.x; dkj[h * 4 + 1] = r4.y;
                        dkj[h * 4 + 2] = r4.z; dkj[h * 4 + 3] = r4.w;
                    }
#pragma unroll
                    for (int m = 0; m < 4; ++m)
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            acc[m][e] = Op::min2(acc[m][e], Op::add(dik[m], dkj[e]));
                    if (big) {
#pragma unroll
                        for (int m = 0; m < 8; ++m)
#pragma unroll
                            for (int e = 0; e < 8; ++e)
                                if (m >= 4 || e >= 4)
                                    acc[m][e] = Op::min2(acc[m][e], Op::add(dik[m], dkj[e]));
                    }
                }
            }
        }
    }
}

}  // namespace tile
}  // namespace apsp

// Single-graph blocked Floyd-Warshall on gfx950 (arXiv:1902.04446, Sec. 4.4 and
// 4.5, Algorithms 3 and 4).  Round r with K = [128 r, min(128 r + 128, n)):
//
//   phase 1  k_phase1        closure of the diagonal block D[K,K] by classic
//                            Floyd-Warshall (Table 1 FloydWarshall), one
//                            workgroup, the block held in registers, pivot
//                            row/column exchanged through LDS;
//   phase 2  k_tiles<..,2>   MinPlus on the block row and block column of K:
//                            D[K,J] = min(D[K,J], D[K,K] (x) D[K,J]),
//                            D[I,K] = min(D[I,K], D[I,K] (x) D[K,K]);
//   phase 3  k_tiles<..,3>   MinPlus on every other block:
//                            D[I,J] = min(D[I,J], D[I,K] (x) D[K,J]).
//
// Phases 2 and 3 are the same 128 x 128 register-blocked min-plus tile
// product; only the workgroup -> tile mapping differs.  A workgroup reads its
// operands before it writes its own tile and no other workgroup of the same
// launch writes those operands, so each phase runs in place.
//
// Precision: every candidate path length is one fp32 (or uint32) addition and
// the minimum is exact, so the result of a phase does not depend on the order
// in which k is visited within it.
#include "apsp_common.h"

namespace apsp {

namespace {

constexpr int TB = kRoundB;  // round width == output tile edge
constexpr int KC = 16;       // k values per LDS stage
constexpr int NT = 256;      // threads per tile workgroup


__device__ __forceinline__ uint4 ld4(const uint32_t *p) {
    return *reinterpret_cast<const uint4 *>(p);
}
__device__ __forceinline__ void st4(uint32_t *p, uint4 v) { *reinterpret_cast<uint4 *>(p) = v; }

// ---------------------------------------------------------------------------
// Input normalisation (first round only): zero diagonal; int32 entries above
// 2^30 (compared as uint32) become 2^30.  Only changed words are written.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_prologue_i32(uint32_t *__restrict__ D, int64_t n,
                                                      int64_t ld) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        uint32_t *p = D + i * ld + j;
        const uint32_t v = *p;
        const uint32_t nv = (i == j) ? 0u : (v > kInfI32 ? kInfI32 : v);
        if (nv != v) *p = nv;
    }
}

__global__ __launch_bounds__(256) void k_diag_zero(uint32_t *__restrict__ D, int64_t n,
                                                   int64_t ld) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) D[i * ld + i] = 0u;
}

// Domain check: int32 must be >= 0; fp32 must be >= 0 or -0 and not NaN.
__global__ __launch_bounds__(256) void k_validate(const uint32_t *__restrict__ D, int64_t n,
                                                  int64_t ld, int is_f32,
                                                  uint32_t *__restrict__ flag) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    bool bad = false;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        const uint32_t v = D[i * ld + j];
        if (is_f32)
            bad |= ((v & 0x7fffffffu) > 0x7f800000u) || ((v >> 31) && v != 0x80000000u);
        else
            bad |= (v >> 31) != 0u;
    }
    if (bad) flag[0] = 1u;  // every writer stores the same value
}

// ---------------------------------------------------------------------------
// Phase 1.  1024 threads; thread t owns row i = t/8 and columns c0..c0+15 of
// the (kw x kw, kw <= 128) diagonal block, in registers.  Step k: the owners
// of row k and of column k publish them to LDS (double-buffered, one barrier
// per step), then every thread applies d_ij = min(d_ij, d_ik + d_kj).  Row k
// and column k do not change during step k (d_kk = 0, weights >= 0), so this
// is exactly the sequential textbook loop.  Entries outside the block are
// padded with the "no edge" value and never stored.
// ---------------------------------------------------------------------------
template <class Op>
__global__ __launch_bounds__(1024) void k_phase1(uint32_t *__restrict__ D, int64_t ld, int64_t kb,
                                                 int kw) {
    __shared__ __align__(16) uint32_t rowbuf[2][TB];
    __shared__ uint32_t colbuf[2][TB];
    const int t = threadIdx.x;
    const int i = t >> 3;
    const int cg = t & 7;
    const int c0 = cg * 16;
    uint32_t *rowp = D + (kb + (i < kw ? i : kw - 1)) * ld + kb;

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
                    for (int w = 0; w < 16; w += 4)
                        *reinterpret_cast<uint4 *>(&rowbuf[s][c0 + w]) =
                            make_uint4(v[w], v[w + 1], v[w + 2], v[w + 3]);
                }
                if (cg == (kk >> 4)) colbuf[s][i] = v[u];
                __syncthreads();
                const uint32_t dik = colbuf[s][i];
#pragma unroll
                for (int w = 0; w < 16; w += 4) {
                    const uint4 rk = *reinterpret_cast<const uint4 *>(&rowbuf[s][c0 + w]);
                    v[w + 0] = Op::min2(v[w + 0], Op::add(dik, rk.x));
                    v[w + 1] = Op::min2(v[w + 1], Op::add(dik, rk.y));
                    v[w + 2] = Op::min2(v[w + 2], Op::add(dik, rk.z));
                    v[w + 3] = Op::min2(v[w + 3], Op::add(dik, rk.w));
                }
            }
        }
    }
    if (i < kw) {
#pragma unroll
        for (int u = 0; u < 16; ++u)
            if (c0 + u < kw) rowp[c0 + u] = v[u];
    }
}

// ---------------------------------------------------------------------------
// Floyd-Warshall closure of a (kw x kw, kw <= 128) diagonal block held in
// registers in the layout of k_tiles (thread (tx, ty) holds rows
// {ty*4 + m, 64 + ty*4 + m}, columns {tx*4 + e, 64 + tx*4 + e}).  Pivot k:
// the 16 threads holding row k and the 16 holding column k publish them to
// LDS (double-buffered, one barrier per pivot), then every thread applies
// d_ij = min(d_ij, d_ik + d_kj) to its 64 entries.  Same operations in the
// same order as k_phase1, so the same bits.  `lds` needs 4 x 128 words.
// ---------------------------------------------------------------------------
template <class Op>
__device__ __forceinline__ void close_block(uint32_t (&acc)[8][8], int kw, int tx, int ty,
                                            uint32_t *lds) {
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
                    for (int m = 0; m < 8; ++m)
#pragma unroll
                        for (int e = 0; e < 8; ++e)
                            acc[m][e] = Op::min2(acc[m][e], Op::add(dik[m], dkj[e]));
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Phases 2 and 3: C = min(C, A (x) B) on a 128 x 128 output tile C at
// (i0, j0), A = D[i0.., K] (128 x kw), B = D[K, j0..] (kw x 128).
//
// 256 threads, thread (tx, ty) = (t % 16, t / 16) holds an 8 x 8 block of C
// in registers: rows {ty*4 + m, 64 + ty*4 + m}, columns {tx*4 + e,
// 64 + tx*4 + e}.  k runs in stages of 16 through double-buffered LDS,
// prefetched into registers one stage ahead.  A is stored in LDS as k-pairs
// (a[i][k], a[i][k+1]) so one min3 folds two candidates:
//     c = min3(c, a[i][k] + b[k][j], a[i][k+1] + b[k+1][j])
// i.e. 2 adds + 1 min3 per 2 updates.  Out-of-range rows, columns and k are
// padded with the "no edge" value, which can never win a minimum.
// ---------------------------------------------------------------------------
template <class Op, int MODE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_tiles(
    uint32_t *__restrict__ D, int64_t ld, int64_t n, int r, int q, int vec, int close_diag) {
    __shared__ uint2 As[2][KC / 2][TB];
    __shared__ uint4 Bs[2][KC][TB / 4];

    int I, J;
    if (MODE == kPanels) {
        int tt = blockIdx.x;
        if (tt < q - 1) {
            I = r;
            J = tt < r ? tt : tt + 1;
        } else {
            tt -= q - 1;
            J = r;
            I = tt < r ? tt : tt + 1;
        }
    } else if (MODE == kNext) {
        // block row r+1 (every column but r), then block column r+1 (every
        // row but r and r+1): the tiles the next round's phases 1 and 2 read
        int tt = blockIdx.x;
        if (tt < q - 1) {
            I = r + 1;
            J = tt < r ? tt : tt + 1;
        } else {
            tt -= q - 1;
            J = r + 1;
            I = tt < r ? tt : tt + 2;
        }
    } else {
        // kAll: every block row/column but r; kRest: every one but r, r+1.
        // Workgroups are dealt round-robin to the 8 XCDs (wg % 8); give each
        // XCD a contiguous range of tiles so tiles sharing panel blocks share
        // that XCD's L2.
        const int skip = (MODE == kRest) ? 2 : 1;
        const int m = q - skip;
        const int T = m * m;
        const int wg = blockIdx.x;
        const int x = wg & 7, s = wg >> 3;
        const int per = T >> 3, rem = T & 7;
        const int tile = x * per + (x < rem ? x : rem) + s;
        const int ti = tile / m, tj = tile - ti * m;
        I = ti < r ? ti : ti + skip;
        J = tj < r ? tj : tj + skip;
    }

    const int64_t i0 = (int64_t)I * TB, j0 = (int64_t)J * TB, kb = (int64_t)r * TB;
    const int kw = (int)((n - kb) < TB ? (n - kb) : TB);
    const int mr = (int)((n - i0) < TB ? (n - i0) : TB);
    const int nc = (int)((n - j0) < TB ? (n - j0) : TB);
    const int t = threadIdx.x;
    const uint32_t PAD = Op::pad();

    // loader roles
    const int ar = t >> 1, ak = (t & 1) * 8;   // A: row ar, k offset ak..ak+7 of a stage
    const int br = t >> 4, bc = (t & 15) * 8;  // B: k row br of a stage, columns bc..bc+7
    const uint32_t *Arow = D + (i0 + (ar < mr ? ar : mr - 1)) * ld + kb;
    const uint32_t *Bbase = D + kb * ld + j0;

    // compute roles
    const int tx = t & 15, ty = t >> 4;

    uint32_t acc[8][8];
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int row = (m >> 2) * 64 + ty * 4 + (m & 3);
        const uint32_t *crow = D + (i0 + (row < mr ? row : mr - 1)) * ld + j0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int col = h * 64 + tx * 4;
            if (vec && row < mr && col + 3 < nc) {
                const uint4 c4 = ld4(crow + col);
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

    uint32_t pa[8], pb[8];
    auto gload = [&](int c) {
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
    };
    auto sstore = [&](int s) {
#pragma unroll
        for (int p = 0; p < 4; ++p) As[s][(ak >> 1) + p][ar] = make_uint2(pa[2 * p], pa[2 * p + 1]);
        Bs[s][br][(bc >> 2) + 0] = make_uint4(pb[0], pb[1], pb[2], pb[3]);
        Bs[s][br][(bc >> 2) + 1] = make_uint4(pb[4], pb[5], pb[6], pb[7]);
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
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const uint2 av = As[s][p][(m >> 2) * 64 + ty * 4 + (m & 3)];
                a0[m] = av.x;
                a1[m] = av.y;
            }
            const uint4 b00 = Bs[s][2 * p][tx], b01 = Bs[s][2 * p][16 + tx];
            const uint4 b10 = Bs[s][2 * p + 1][tx], b11 = Bs[s][2 * p + 1][16 + tx];
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
        if (c + 1 < nch) sstore(s ^ 1);
        __syncthreads();
    }

    // Phase 1 of round r+1, fused: the workgroup that just produced diagonal
    // block r+1 closes it in registers before storing it (classic
    // Floyd-Warshall over its pivots; see close_block).
    if (MODE == kNext && close_diag && I == r + 1 && J == r + 1)
        close_block<Op>(acc, mr, tx, ty, reinterpret_cast<uint32_t *>(&As[0][0][0]));

#pragma unroll
    for (int m = 0; m < 8; ++m) {
        const int row = (m >> 2) * 64 + ty * 4 + (m & 3);
        if (row >= mr) continue;
        uint32_t *crow = D + (i0 + row) * ld + j0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int col = h * 64 + tx * 4;
            if (vec && col + 3 < nc) {
                st4(crow + col, make_uint4(acc[m][h * 4 + 0], acc[m][h * 4 + 1],
                                           acc[m][h * 4 + 2], acc[m][h * 4 + 3]));
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (col + e < nc) crow[col + e] = acc[m][h * 4 + e];
            }
        }
    }
}

inline bool aligned16(const void *p, int64_t ld) {
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0 && (ld & 3) == 0;
}

inline unsigned grid_rows(int64_t n) { return (unsigned)(n < 8192 ? n : 8192); }

template <class Op>
void launch_tiles(int set, uint32_t *D, int64_t n, int64_t ld, int r, int q, int vec, int close,
                  hipStream_t s, unsigned grid) {
    switch (set) {
    case kPanels:
        hipLaunchKernelGGL((k_tiles<Op, kPanels>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close);
        break;
    case kAll:
        hipLaunchKernelGGL((k_tiles<Op, kAll>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close);
        break;
    case kNext:
        hipLaunchKernelGGL((k_tiles<Op, kNext>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close);
        break;
    default:
        hipLaunchKernelGGL((k_tiles<Op, kRest>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close);
        break;
    }
}

}  // namespace

hipError_t launch_prologue(uint32_t *D, int64_t n, int64_t ld, int dtype, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (dtype == 0) {
        dim3 grid((unsigned)((n + 255) / 256), grid_rows(n));
        hipLaunchKernelGGL(k_prologue_i32, grid, dim3(256), 0, s, D, n, ld);
    } else {
        hipLaunchKernelGGL(k_diag_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, D, n,
                           ld);
    }
    return hipGetLastError();
}

hipError_t launch_validate(const uint32_t *D, int64_t n, int64_t ld, int dtype, uint32_t *flag,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256), grid_rows(n));
    hipLaunchKernelGGL(k_validate, grid, dim3(256), 0, s, D, n, ld, dtype == 1 ? 1 : 0, flag);
    return hipGetLastError();
}

int64_t num_rounds(int64_t n) { return (n + TB - 1) / TB; }

int64_t tile_count(int64_t n, int64_t r, int set) {
    const int64_t q = num_rounds(n);
    if (r < 0 || r >= q) return 0;
    switch (set) {
    case kPanels: return 2 * (q - 1);
    case kAll: return (q - 1) * (q - 1);
    case kNext: return (r + 1 < q) ? 2 * q - 3 : 0;
    case kRest: return (r + 1 < q) ? (q - 2) * (q - 2) : 0;
    default: return 0;
    }
}

hipError_t launch_phase1(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, hipStream_t s) {
    const int64_t kb = r * TB;
    if (kb >= n) return hipSuccess;
    const int kw = (int)((n - kb) < TB ? (n - kb) : TB);
    if (dtype == 0)
        hipLaunchKernelGGL(k_phase1<OpI32>, dim3(1), dim3(1024), 0, s, D, ld, kb, kw);
    else
        hipLaunchKernelGGL(k_phase1<OpF32>, dim3(1), dim3(1024), 0, s, D, ld, kb, kw);
    return hipGetLastError();
}

hipError_t launch_tile_set(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, int set,
                           hipStream_t s, bool close_next_diag) {
    const int64_t count = tile_count(n, r, set);
    if (count <= 0) return hipSuccess;
    const int q = (int)num_rounds(n);
    const int vec = aligned16(D, ld) ? 1 : 0;
    const int close = (set == kNext && close_next_diag) ? 1 : 0;
    if (dtype == 0)
        launch_tiles<OpI32>(set, D, n, ld, (int)r, q, vec, close, s, (unsigned)count);
    else
        launch_tiles<OpF32>(set, D, n, ld, (int)r, q, vec, close, s, (unsigned)count);
    return hipGetLastError();
}

}  // namespace apsp

// Single-graph blocked Floyd-Warshall on gfx950 (arXiv:1902.04446, Sec. 4.4 and
// 4.5, Algorithms 3 and 4).  Round r with K = [128 r, min(128 r + 128, n)):
//
//   phase 1  k_phase1        closure of the diagonal block D[K,K] by classic
//                            Floyd-Warshall (Table 1 FloydWarshall), one
//                            workgroup, the block held in registers, pivot
//                            row/column exchanged through LDS;
//   phase 2  k_tiles<kPanels>  MinPlus on the block row and block column of K:
//                            D[K,J] = min(D[K,J], D[K,K] (x) D[K,J]),
//                            D[I,K] = min(D[I,K], D[I,K] (x) D[K,K]);
//   phase 3  k_tiles<kAll>     MinPlus on every other block:
//            (or kNext+kRest)  D[I,J] = min(D[I,J], D[I,K] (x) D[K,J]).
//
// Phases 2 and 3 are the same 128 x 128 register-blocked min-plus tile
// product; only the workgroup -> tile mapping differs.  A workgroup reads its
// operands before it writes its own tile and no other workgroup of the same
// launch writes those operands, so each phase runs in place.
//
// Precision: every candidate path length is one fp32 (or uint32) addition and
// the minimum is exact, so the result of a phase does not depend on the order
// in which k is visited within it.
#include <algorithm>

#include "apsp_tile.h"
#include "apsp_tilemap.h"

namespace apsp {

namespace {

using tile::NT;
using tile::TB;

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
__device__ __forceinline__ void phase1_block(uint32_t *__restrict__ D, int64_t ld, int64_t kb,
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

template <class Op>
__global__ __launch_bounds__(1024) void k_phase1(uint32_t *__restrict__ D, int64_t ld, int64_t kb,
                                                 int kw) {
    tile::chain_priority();
    phase1_block<Op>(D, ld, kb, kw);
}

// int32 matrix held as fp32 bits (OpI32F's form) when *wmax allows it, as
// uint32 otherwise (converted by launch_conv_i32 before the first round).
__global__ __launch_bounds__(1024) void k_phase1_conv(uint32_t *__restrict__ D, int64_t ld,
                                                      int64_t n, int64_t kb, int kw,
                                                      const uint32_t *__restrict__ wmax) {
    tile::chain_priority();
    if (int_exact_in_f32(n, *wmax))
        phase1_block<OpF32>(D, ld, kb, kw);
    else
        phase1_block<OpI32>(D, ld, kb, kw);
}

// int32 <-> the fp32 bits OpI32F computes on, in place, when *wmax allows
// the fp32 pipe (else nothing): to_f32 v -> (float)min(v, 2^30), back
// f -> min((uint32)f, 2^30).  Thread = column, rows strided by the grid's y.
__global__ __launch_bounds__(256) void k_conv_i32(uint32_t *__restrict__ D, int64_t n, int64_t ld,
                                                  const uint32_t *__restrict__ wmax, int to_f32) {
    if (!int_exact_in_f32(n, *wmax)) return;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
        uint32_t *p = D + i * ld + j;
        *p = to_f32 ? OpI32F::norm(*p) : OpI32F::out(*p);
    }
}

// ---------------------------------------------------------------------------
// Phases 2 and 3: one workgroup per 128 x 128 output tile C at (i0, j0),
// C = min(C, A (x) B) with A = D[i0.., K] and B = D[K, j0..]
// (tile::minplus_tile; 8 x 8 registers per thread, k-paired min3).  MODE
// selects the tile set of the launch (apsp_common.h); the workgroup -> tile
// maps (apsp_tilemap.h) are bijections onto each set.
// ---------------------------------------------------------------------------
template <int MODE>
__device__ __forceinline__ void tile_of(int r, int q, int row_lo, int row_hi, int &I, int &J) {
    tilemap::tile_of<MODE>((int)blockIdx.x, r, q, row_lo, row_hi, I, J);
}

// NORM converts on load and store (OpI32F: int32 storage, fp32 arithmetic).
template <class Op, int MODE, bool NORM>
__device__ __forceinline__ void tile_update(uint32_t *D, int64_t ld, int64_t n, int r, int I,
                                            int J, bool vec, bool close_diag, tile::Lds &L) {
    const int64_t i0 = (int64_t)I * TB, j0 = (int64_t)J * TB, kb = (int64_t)r * TB;
    const int kw = (int)((n - kb) < TB ? (n - kb) : TB);
    const int mr = (int)((n - i0) < TB ? (n - i0) : TB);
    const int nc = (int)((n - j0) < TB ? (n - j0) : TB);

    uint32_t acc[8][8];
    tile::load_acc<Op, NORM>(acc, D, ld, i0, j0, mr, nc, vec);
    tile::minplus_tile<Op, NORM>(acc, D, ld, i0, j0, kb, mr, nc, kw, vec, L);
    // Phase 1 of round r+1, fused: the workgroup that just produced diagonal
    // block r+1 closes it in registers before storing it.
    if ((MODE == kNext || MODE == kAll) && close_diag && I == r + 1 && J == r + 1)
        tile::close_block<Op>(acc, mr, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
    tile::store_acc<Op>(acc, D, ld, i0, j0, mr, nc, vec);
}

template <class Op, int MODE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_tiles(
    uint32_t *__restrict__ D, int64_t ld, int64_t n, int r, int q, int vec, int close_diag,
    int row_lo, int row_hi) {
    __shared__ tile::Lds L;
    if (MODE == kPanels || MODE == kNext) tile::chain_priority();
    int I, J;
    tile_of<MODE>(r, q, row_lo, row_hi, I, J);
    tile_update<Op, MODE, false>(D, ld, n, r, I, J, vec != 0, close_diag != 0, L);
}

// int32: on the fp32 pipe (OpI32F, bit-identical) when the matrix's largest
// finite entry *wmax allows it, else in uint32.
// CONV: the matrix is held as fp32 bits when *wmax allows the fp32 pipe
// (launch_conv_i32), so those tiles compute as OpF32 with no conversion.
template <int MODE, bool CONV>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_tiles_i32(
    uint32_t *__restrict__ D, int64_t ld, int64_t n, int r, int q, int vec, int close_diag,
    int row_lo, int row_hi, const uint32_t *__restrict__ wmax) {
    __shared__ tile::Lds L;
    if (MODE == kPanels || MODE == kNext) tile::chain_priority();
    int I, J;
    tile_of<MODE>(r, q, row_lo, row_hi, I, J);
    if (int_exact_in_f32(n, *wmax)) {
        if (CONV)
            tile_update<OpF32, MODE, false>(D, ld, n, r, I, J, vec != 0, close_diag != 0, L);
        else
            tile_update<OpI32F, MODE, true>(D, ld, n, r, I, J, vec != 0, close_diag != 0, L);
    } else {
        tile_update<OpI32, MODE, false>(D, ld, n, r, I, J, vec != 0, close_diag != 0, L);
    }
}

__global__ void k_zero_word(uint32_t *w) { *w = 0u; }

// *wmax = max(*wmax, largest finite off-diagonal entry): thread = column,
// rows strided by the grid's y extent; one atomic per workgroup.
__global__ __launch_bounds__(256) void k_wmax(const uint32_t *__restrict__ D, int64_t n,
                                              int64_t ld, uint32_t *wmax) {
    __shared__ uint32_t part[4];
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    uint32_t m = 0;
    if (j < n)
        for (int64_t i = blockIdx.y; i < n; i += gridDim.y) {
            const uint32_t v = D[i * ld + j];
            if (v < kInfI32 && i != j && v > m) m = v;
        }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)m, off);
        m = o > m ? o : m;
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = part[0];
        for (int w = 1; w < 4; ++w) m = part[w] > m ? part[w] : m;
        if (m > 0) atomicMax(wmax, m);
    }
}

inline bool aligned16(const void *p, int64_t ld) {
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0 && (ld & 3) == 0;
}

inline unsigned grid_rows(int64_t n) { return (unsigned)(n < 8192 ? n : 8192); }

template <bool CONV>
void launch_tiles_i32_as(int set, uint32_t *D, int64_t n, int64_t ld, int r, int q, int vec,
                         int close, int lo, int hi, const uint32_t *wmax, hipStream_t s,
                         unsigned grid) {
    switch (set) {
    case kPanels:
        hipLaunchKernelGGL((k_tiles_i32<kPanels, CONV>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close, lo, hi, wmax);
        break;
    case kAll:
        hipLaunchKernelGGL((k_tiles_i32<kAll, CONV>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close, lo, hi, wmax);
        break;
    case kNext:
        hipLaunchKernelGGL((k_tiles_i32<kNext, CONV>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close, lo, hi, wmax);
        break;
    default:
        hipLaunchKernelGGL((k_tiles_i32<kRest, CONV>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close, lo, hi, wmax);
        break;
    }
}

void launch_tiles_i32(bool conv, int set, uint32_t *D, int64_t n, int64_t ld, int r, int q,
                      int vec, int close, int lo, int hi, const uint32_t *wmax, hipStream_t s,
                      unsigned grid) {
    if (conv)
        launch_tiles_i32_as<true>(set, D, n, ld, r, q, vec, close, lo, hi, wmax, s, grid);
    else
        launch_tiles_i32_as<false>(set, D, n, ld, r, q, vec, close, lo, hi, wmax, s, grid);
}

template <class Op>
void launch_tiles(int set, uint32_t *D, int64_t n, int64_t ld, int r, int q, int vec, int close,
                  int lo, int hi, hipStream_t s, unsigned grid) {
    switch (set) {
    case kPanels:
        hipLaunchKernelGGL((k_tiles<Op, kPanels>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close, lo, hi);
        break;
    case kAll:
        hipLaunchKernelGGL((k_tiles<Op, kAll>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close, lo, hi);
        break;
    case kNext:
        hipLaunchKernelGGL((k_tiles<Op, kNext>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close, lo, hi);
        break;
    default:
        hipLaunchKernelGGL((k_tiles<Op, kRest>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close, lo, hi);
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
    return tilemap::tile_count(q, r, set, 0, q);
}

hipError_t launch_conv_i32(uint32_t *D, int64_t n, int64_t ld, const uint32_t *wmax, bool to_f32,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256), grid_rows(n));
    hipLaunchKernelGGL(k_conv_i32, grid, dim3(256), 0, s, D, n, ld, wmax, to_f32 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_phase1(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, hipStream_t s,
                         const uint32_t *wmax) {
    const int64_t kb = r * TB;
    if (kb >= n) return hipSuccess;
    const int kw = (int)((n - kb) < TB ? (n - kb) : TB);
    if (dtype == kI32AsF32)
        hipLaunchKernelGGL(k_phase1_conv, dim3(1), dim3(1024), 0, s, D, ld, n, kb, kw, wmax);
    else if (dtype == 0)
        hipLaunchKernelGGL(k_phase1<OpI32>, dim3(1), dim3(1024), 0, s, D, ld, kb, kw);
    else
        hipLaunchKernelGGL(k_phase1<OpF32>, dim3(1), dim3(1024), 0, s, D, ld, kb, kw);
    return hipGetLastError();
}

hipError_t launch_tile_set(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, int set,
                           hipStream_t s, bool close_next_diag, const uint32_t *wmax) {
    const int64_t count = tile_count(n, r, set);
    if (count <= 0) return hipSuccess;
    const int q = (int)num_rounds(n);
    const int vec = aligned16(D, ld) ? 1 : 0;
    const int close = ((set == kNext || set == kAll) && close_next_diag) ? 1 : 0;
    if ((dtype == 0 || dtype == kI32AsF32) && wmax)
        launch_tiles_i32(dtype == kI32AsF32, set, D, n, ld, (int)r, q, vec, close, 0, q, wmax, s,
                         (unsigned)count);
    else if (dtype == 0)
        launch_tiles<OpI32>(set, D, n, ld, (int)r, q, vec, close, 0, q, s, (unsigned)count);
    else
        launch_tiles<OpF32>(set, D, n, ld, (int)r, q, vec, close, 0, q, s, (unsigned)count);
    return hipGetLastError();
}

hipError_t launch_wmax(const uint32_t *D, int64_t n, int64_t ld, uint32_t *wmax, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_word, dim3(1), dim3(1), 0, s, wmax);
    if (n > 0) {
        // about 4096 workgroups, so about as many atomics on the one word
        const unsigned gx = (unsigned)((n + 255) / 256);
        const unsigned gy = gx >= 4096 ? 1u : (unsigned)std::min<int64_t>(4096 / gx, n);
        hipLaunchKernelGGL(k_wmax, dim3(gx, gy), dim3(256), 0, s, D, n, ld, wmax);
    }
    return hipGetLastError();
}

int64_t rest_rows_count(int64_t n, int64_t r, int64_t lo, int64_t hi) {
    return tilemap::tile_count(num_rounds(n), r, kRest, lo, hi);
}

hipError_t launch_rest_rows(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, int64_t lo,
                            int64_t hi, hipStream_t s, const uint32_t *wmax) {
    const int64_t count = rest_rows_count(n, r, lo, hi);
    if (count <= 0) return hipSuccess;
    const int q = (int)num_rounds(n);
    const int vec = aligned16(D, ld) ? 1 : 0;
    if ((dtype == 0 || dtype == kI32AsF32) && wmax)
        launch_tiles_i32(dtype == kI32AsF32, kRest, D, n, ld, (int)r, q, vec, 0, (int)lo, (int)hi,
                         wmax, s, (unsigned)count);
    else if (dtype == 0)
        launch_tiles<OpI32>(kRest, D, n, ld, (int)r, q, vec, 0, (int)lo, (int)hi, s, (unsigned)count);
    else
        launch_tiles<OpF32>(kRest, D, n, ld, (int)r, q, vec, 0, (int)lo, (int)hi, s, (unsigned)count);
    return hipGetLastError();
}

}  // namespace apsp

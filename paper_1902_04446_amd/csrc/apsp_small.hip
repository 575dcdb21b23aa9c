// Width-64 rounds of the single-graph solver, for small matrices
// (arXiv:1902.04446, Sec. 4.4/4.5, Algorithms 3 and 4 with b = 64; Sec. 4
// leaves b to the user or a tuner).
//
// Below a few thousand vertices a solve is a chain of dependent launches
// (phase 2 of round r, then the tiles of block row/column r+1 with the
// closure of diagonal block r+1), each run by few workgroups: a round costs
// the chain's latency, not its work.  Rounds of 64 halve the chain's work
// per round (a 64 x 64 x 64 tile update, a 64-pivot closure) for twice the
// rounds, and the chain shortens overall.  Same schedule as the 128-wide
// single rounds (apsp_runtime.hip: one-round lookahead, the rest of phase 3
// on a helper stream); the tiles are tile64's: 256 threads, 4 x 4 registers
// each, the 64-wide k range staged in LDS at once.
#include "apsp_tile.h"
#include "apsp_tile64.h"
#include "apsp_tilemap.h"

namespace apsp {

namespace {

using tile64::T64;

template <class Op, int MODE>
__device__ __forceinline__ void tile64_update(uint32_t *D, int64_t ld, int64_t n, int r, int I,
                                              int J, bool vec, bool close_diag, tile64::Lds64 &L) {
    const int kb = r * T64, i0 = I * T64, j0 = J * T64;
    const int kw = (int)((n - kb) < T64 ? (n - kb) : T64);
    const int mr = (int)((n - i0) < T64 ? (n - i0) : T64);
    const int nc = (int)((n - j0) < T64 ? (n - j0) : T64);
    uint32_t acc[4][4];
    tile64::load64<Op>(acc, D, ld, i0, j0, mr, nc, vec);
    tile64::update64<Op>(acc, D, ld, i0, j0, kb, mr, nc, kw, vec, L);
    // phase 1 of round r+1, fused into the workgroup that produced its block
    if ((MODE == kNext || MODE == kAll) && close_diag && I == r + 1 && J == r + 1)
        tile64::close64_pairs<Op>(acc, mr, L);
    tile64::store64<Op>(acc, D, ld, i0, j0, mr, nc, vec);
}

template <class Op, int MODE>
__global__ __launch_bounds__(256) void k_tiles64(uint32_t *__restrict__ D, int64_t ld, int64_t n,
                                                 int r, int q, int vec, int close_diag,
                                                 int row_lo, int row_hi) {
    __shared__ tile64::Lds64 L;
    if (MODE == kPanels || MODE == kNext) tile::chain_priority();
    int I, J;
    tilemap::tile_of<MODE>((int)blockIdx.x, r, q, row_lo, row_hi, I, J);
    tile64_update<Op, MODE>(D, ld, n, r, I, J, vec != 0, close_diag != 0, L);
}

// int32: the fp32 pipe (OpI32F, bit-identical) when *wmax allows it.
template <int MODE>
__global__ __launch_bounds__(256) void k_tiles64_i32(uint32_t *__restrict__ D, int64_t ld,
                                                     int64_t n, int r, int q, int vec,
                                                     int close_diag, int row_lo, int row_hi,
                                                     const uint32_t *__restrict__ wmax) {
    __shared__ tile64::Lds64 L;
    if (MODE == kPanels || MODE == kNext) tile::chain_priority();
    int I, J;
    tilemap::tile_of<MODE>((int)blockIdx.x, r, q, row_lo, row_hi, I, J);
    if (int_exact_in_f32(n, *wmax))
        tile64_update<OpI32F, MODE>(D, ld, n, r, I, J, vec != 0, close_diag != 0, L);
    else
        tile64_update<OpI32, MODE>(D, ld, n, r, I, J, vec != 0, close_diag != 0, L);
}

// Phase 1 of round r: Floyd-Warshall closure of diagonal block r, pivots
// ascending (tile64::close64), one workgroup.
template <class Op>
__global__ __launch_bounds__(256) void k_phase1_64(uint32_t *__restrict__ D, int64_t ld, int64_t n,
                                                   int r, int vec) {
    __shared__ tile64::Lds64 L;
    tile::chain_priority();
    const int kb = r * T64;
    const int kw = (int)((n - kb) < T64 ? (n - kb) : T64);
    uint32_t acc[4][4];
    tile64::load64<Op>(acc, D, ld, kb, kb, kw, kw, vec);
    tile64::close64_pairs<Op>(acc, kw, L);
    tile64::store64<Op>(acc, D, ld, kb, kb, kw, kw, vec);
}

template <class Op, int MODE>
void launch_op(dim3 grid, hipStream_t s, uint32_t *D, int64_t ld, int64_t n, int r, int q, int vec,
               int close, int lo, int hi) {
    hipLaunchKernelGGL((k_tiles64<Op, MODE>), grid, dim3(256), 0, s, D, ld, n, r, q, vec, close,
                       lo, hi);
}

template <int MODE>
void launch_mode(int dtype, const uint32_t *wmax, dim3 grid, hipStream_t s, uint32_t *D,
                 int64_t ld, int64_t n, int r, int q, int vec, int close, int lo, int hi) {
    if (dtype == 0 && wmax)
        hipLaunchKernelGGL((k_tiles64_i32<MODE>), grid, dim3(256), 0, s, D, ld, n, r, q, vec,
                           close, lo, hi, wmax);
    else if (dtype == 0)
        launch_op<OpI32, MODE>(grid, s, D, ld, n, r, q, vec, close, lo, hi);
    else
        launch_op<OpF32, MODE>(grid, s, D, ld, n, r, q, vec, close, lo, hi);
}

}  // namespace

int64_t num_rounds64(int64_t n) { return (n + T64 - 1) / T64; }

hipError_t launch_phase1_64(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                            hipStream_t s) {
    if (r * T64 >= n) return hipSuccess;
    const int vec = ((reinterpret_cast<uintptr_t>(D) & 15u) == 0 && (ld & 3) == 0) ? 1 : 0;
    if (dtype == 0)
        hipLaunchKernelGGL(k_phase1_64<OpI32>, dim3(1), dim3(256), 0, s, D, ld, n, (int)r, vec);
    else
        hipLaunchKernelGGL(k_phase1_64<OpF32>, dim3(1), dim3(256), 0, s, D, ld, n, (int)r, vec);
    return hipGetLastError();
}

hipError_t launch_tile_set64(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, int set,
                             hipStream_t s, bool close_next_diag, const uint32_t *wmax,
                             int64_t lo, int64_t hi) {
    const int64_t q = num_rounds64(n);
    if (set != kRest) {
        lo = 0;
        hi = q;
    }
    const int64_t count = tilemap::tile_count(q, r, set, lo, hi);
    if (count <= 0) return hipSuccess;
    const int vec = ((reinterpret_cast<uintptr_t>(D) & 15u) == 0 && (ld & 3) == 0) ? 1 : 0;
    const int close = ((set == kNext || set == kAll) && close_next_diag) ? 1 : 0;
    const dim3 grid((unsigned)count);
    switch (set) {
    case kPanels:
        launch_mode<kPanels>(dtype, wmax, grid, s, D, ld, n, (int)r, (int)q, vec, close, (int)lo, (int)hi);
        break;
    case kAll:
        launch_mode<kAll>(dtype, wmax, grid, s, D, ld, n, (int)r, (int)q, vec, close, (int)lo, (int)hi);
        break;
    case kNext:
        launch_mode<kNext>(dtype, wmax, grid, s, D, ld, n, (int)r, (int)q, vec, close, (int)lo, (int)hi);
        break;
    default:
        launch_mode<kRest>(dtype, wmax, grid, s, D, ld, n, (int)r, (int)q, vec, close, (int)lo, (int)hi);
        break;
    }
    return hipGetLastError();
}

}  // namespace apsp

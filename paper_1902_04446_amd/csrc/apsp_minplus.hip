// Standalone min-plus product (arXiv:1902.04446, Table 1: MatProd is the
// (min, +) product, MinPlus is MatProd followed by MatMin) and the
// repeated-squaring APSP solver built on it (Sec. 4.2, Algorithm 1: A^n by
// repeated min-plus squaring).
//
// One workgroup per 128 x 128 output tile, the same register-blocked tile
// update as the blocked solver (tile::minplus_tile_ab), here over the whole
// k extent of the product.  Output tiles are dealt so that each XCD gets one
// contiguous range of tiles (row-major), which share rows of A in its L2.
#include "apsp_tile.h"

namespace apsp {

namespace {

using tile::NT;
using tile::TB;

template <class Op>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_minplus(
    uint32_t *__restrict__ C, int64_t ldc, const uint32_t *__restrict__ A, int64_t lda,
    const uint32_t *__restrict__ B, int64_t ldb, int64_t m, int64_t n, int64_t k, int tiles_n,
    int tiles, int vec_c, int vec_ab, int accumulate) {
    __shared__ tile::Lds L;
    const int wg = blockIdx.x;
    const int x = wg & 7, s = wg >> 3;
    const int per = tiles >> 3, rem = tiles & 7;
    const int id = x * per + (x < rem ? x : rem) + s;
    const int ti = id / tiles_n, tj = id - ti * tiles_n;
    const int64_t i0 = (int64_t)ti * TB, j0 = (int64_t)tj * TB;
    const int mr = (int)((m - i0) < TB ? (m - i0) : TB);
    const int nc = (int)((n - j0) < TB ? (n - j0) : TB);

    uint32_t acc[8][8];
    if (accumulate) {
        tile::load_acc<Op, false>(acc, C, ldc, i0, j0, mr, nc, vec_c != 0);
    } else {
#pragma unroll
        for (int a = 0; a < 8; ++a)
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[a][e] = Op::pad();
    }
    tile::minplus_tile_ab<Op, false>(acc, A, lda, B, ldb, i0, j0, mr, nc, (int)k, vec_ab != 0, L);
    tile::store_acc<Op>(acc, C, ldc, i0, j0, mr, nc, vec_c != 0);
}

bool aligned_rows(const void *p, int64_t ld) {
    return (reinterpret_cast<uintptr_t>(p) & 15u) == 0 && (ld & 3) == 0;
}

}  // namespace

hipError_t launch_minplus(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                          const uint32_t *B, int64_t ldb, int64_t m, int64_t n, int64_t k,
                          int dtype, bool accumulate, hipStream_t s) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const int64_t tm = (m + TB - 1) / TB, tn = (n + TB - 1) / TB;
    const int tiles = (int)(tm * tn);
    const int vec_c = aligned_rows(C, ldc) ? 1 : 0;
    const int vec_ab = (aligned_rows(A, lda) && aligned_rows(B, ldb)) ? 1 : 0;
    const dim3 grid((unsigned)tiles);
    if (dtype == 0)
        hipLaunchKernelGGL(k_minplus<OpI32>, grid, dim3(NT), 0, s, C, ldc, A, lda, B, ldb, m, n, k,
                           (int)tn, tiles, vec_c, vec_ab, accumulate ? 1 : 0);
    else
        hipLaunchKernelGGL(k_minplus<OpF32>, grid, dim3(NT), 0, s, C, ldc, A, lda, B, ldb, m, n, k,
                           (int)tn, tiles, vec_c, vec_ab, accumulate ? 1 : 0);
    return hipGetLastError();
}

}  // namespace apsp

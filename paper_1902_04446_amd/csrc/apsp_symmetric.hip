// Symmetric variant of the blocked method for undirected graphs.  The paper
// stores only the upper-triangular blocks and transposes on demand (Sec. 4):
// with A symmetric, every round keeps D symmetric, so only blocks (I, J)
// with I <= J are updated:
//
//   phase 2  row panel (r, J), J > r: D_rJ = min(D_rJ, D_rr (x) D_rJ);
//            column panel (I, r), I < r: D_Ir = min(D_Ir, D_Ir (x) D_rr);
//   phase 3  (I, J), I <= J, I, J != r: D_IJ = min(D_IJ, D_Ir (x) D_rJ), where
//            D_Ir for I > r is read as the transpose of (r, I) and D_rJ for
//            J < r as the transpose of (J, r) (tile::minplus_tile_ab, TA/TB);
//
// and the strict lower triangle is filled from the upper one at the end (and
// once before the first round, so the input's lower triangle is never read).
// Every candidate D_Ik + D_kJ of block (J, I) in the full method equals
// D_kJ + D_Ik here (fp32 addition is commutative), so the result is the full
// method's, bit for bit, at about half its phase-2 and phase-3 work.
#include "apsp_tile.h"

namespace apsp {

namespace {

using tile::NT;
using tile::TB;

template <class Op>
__device__ __forceinline__ void sym_product(uint32_t (&acc)[8][8], uint32_t *D, int64_t ld, int I,
                                            int J, int r, int64_t i0, int64_t j0, int64_t kb,
                                            int mr, int nc, int kw, bool vec, tile::Lds &L) {
    const bool ta = I > r, tb = J < r;
    // direct A = D[i0.., kb..]; transposed A from block (r, I) = D[kb.., i0..]
    // direct B = D[kb.., j0..]; transposed B from block (J, r) = D[j0.., kb..]
    if (!ta && !tb)
        tile::minplus_tile_ab<Op, false, false, false>(acc, D + kb, ld, D + kb * ld, ld, i0, j0,
                                                       mr, nc, kw, vec, L);
    else if (ta && !tb)
        tile::minplus_tile_ab<Op, false, true, false>(acc, D + kb * ld, ld, D + kb * ld, ld, i0, j0,
                                                      mr, nc, kw, vec, L);
    else if (!ta && tb)
        tile::minplus_tile_ab<Op, false, false, true>(acc, D + kb, ld, D + kb, ld, i0, j0, mr, nc,
                                                      kw, vec, L);
    else
        tile::minplus_tile_ab<Op, false, true, true>(acc, D + kb * ld, ld, D + kb, ld, i0, j0, mr,
                                                     nc, kw, vec, L);
}

// MODE 0: the q-1 upper panel blocks of round r; MODE 1: the upper blocks
// outside block row/column r, with the closure of diagonal block r+1 fused.
template <class Op, int MODE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_sym(
    uint32_t *__restrict__ D, int64_t ld, int64_t n, int r, int q, int vec, int close_diag) {
    __shared__ tile::Lds L;
    int I, J;
    if (MODE == 0) {
        const int t = blockIdx.x;
        if (t < q - 1 - r) {
            I = r;
            J = r + 1 + t;
        } else {
            I = t - (q - 1 - r);
            J = r;
        }
    } else {
        // upper triangle (a <= b) of the (q-1) x (q-1) grid without block r,
        // row-major; each XCD (wg % 8) gets one contiguous range of it
        const int m = q - 1;
        const int T = m * (m + 1) / 2;
        const int wg = blockIdx.x;
        const int x = wg & 7, s = wg >> 3;
        const int per = T >> 3, rem = T & 7;
        int id = x * per + (x < rem ? x : rem) + s;
        int a = 0;
        while (id >= m - a) {  // row a holds m - a entries
            id -= m - a;
            ++a;
        }
        const int b = a + id;
        I = a < r ? a : a + 1;
        J = b < r ? b : b + 1;
    }
    const int64_t i0 = (int64_t)I * TB, j0 = (int64_t)J * TB, kb = (int64_t)r * TB;
    const int kw = (int)((n - kb) < TB ? (n - kb) : TB);
    const int mr = (int)((n - i0) < TB ? (n - i0) : TB);
    const int nc = (int)((n - j0) < TB ? (n - j0) : TB);
    uint32_t acc[8][8];
    tile::load_acc<Op, false>(acc, D, ld, i0, j0, mr, nc, vec);
    sym_product<Op>(acc, D, ld, I, J, r, i0, j0, kb, mr, nc, kw, vec, L);
    if (MODE == 1 && close_diag && I == r + 1 && J == r + 1)
        tile::close_block<Op>(acc, mr, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
    tile::store_acc<Op>(acc, D, ld, i0, j0, mr, nc, vec);
}

// Fill the strict lower triangle from the upper one, in 64 x 64 blocks:
// block (a, b), a <= b, is transposed into (b, a) through LDS; a block on the
// diagonal copies only its strict upper part into its strict lower part.
__global__ __launch_bounds__(256) void k_mirror(uint32_t *__restrict__ D, int64_t ld, int64_t n,
                                                int nb) {
    __shared__ uint32_t tileb[64][65];
    int id = blockIdx.x, a = 0;
    while (id >= nb - a) {  // row a of the upper triangle has nb - a blocks (b = a .. nb-1)
        id -= nb - a;
        ++a;
    }
    const int b = a + id;
    const int64_t r0 = (int64_t)a * 64, c0 = (int64_t)b * 64;
    const int t = threadIdx.x;
    const int tc = t & 63, tr = t >> 6;  // 4 rows per pass
    for (int i = tr; i < 64; i += 4) {
        const int64_t row = r0 + i, col = c0 + tc;
        if (row < n && col < n) tileb[i][tc] = D[row * ld + col];
    }
    __syncthreads();
    for (int i = tr; i < 64; i += 4) {
        const int64_t row = c0 + i, col = r0 + tc;  // (b-block row i, a-block column tc)
        if (row < n && col < n && (a != b || i > tc)) D[row * ld + col] = tileb[tc][i];
    }
}

template <class Op>
void launch_sym(int mode, uint32_t *D, int64_t ld, int64_t n, int r, int q, int vec, int close,
                hipStream_t s, unsigned grid) {
    if (mode == 0)
        hipLaunchKernelGGL((k_sym<Op, 0>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close);
    else
        hipLaunchKernelGGL((k_sym<Op, 1>), dim3(grid), dim3(NT), 0, s, D, ld, n, r, q, vec, close);
}

}  // namespace

hipError_t run_symmetric(uint32_t *D, int64_t n, int64_t ld, int dtype, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nb = (int)((n + 63) / 64);
    const dim3 mgrid((unsigned)((int64_t)nb * (nb + 1) / 2));
    hipError_t e = launch_prologue(D, n, ld, dtype, s);
    // the input's lower triangle is not read: make the matrix symmetric first
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mirror, mgrid, dim3(256), 0, s, D, ld, n, nb);
        e = hipGetLastError();
    }
    const int q = (int)((n + TB - 1) / TB);
    const int vec = ((reinterpret_cast<uintptr_t>(D) & 15u) == 0 && (ld & 3) == 0) ? 1 : 0;
    bool closed = false;
    for (int r = 0; r < q && e == hipSuccess; ++r) {
        if (!closed) e = launch_phase1(D, n, ld, dtype, r, s);
        closed = false;
        if (q > 1 && e == hipSuccess) {
            const unsigned g2 = (unsigned)(q - 1);
            const unsigned g3 = (unsigned)((q - 1) * q / 2);
            const int fuse = r + 1 < q ? 1 : 0;
            if (dtype == 0) {
                launch_sym<OpI32>(0, D, ld, n, r, q, vec, 0, s, g2);
                launch_sym<OpI32>(1, D, ld, n, r, q, vec, fuse, s, g3);
            } else {
                launch_sym<OpF32>(0, D, ld, n, r, q, vec, 0, s, g2);
                launch_sym<OpF32>(1, D, ld, n, r, q, vec, fuse, s, g3);
            }
            closed = fuse != 0;
            e = hipGetLastError();
        }
    }
    if (e == hipSuccess) {  // blocks below the diagonal were not updated
        hipLaunchKernelGGL(k_mirror, mgrid, dim3(256), 0, s, D, ld, n, nb);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace apsp

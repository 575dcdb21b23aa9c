// Symmetric variant of the blocked method for undirected graphs.  The paper
// stores only the upper-triangular blocks and transposes on demand (Sec. 4):
// with A symmetric, every round keeps D symmetric, so only blocks (I, J)
// with I <= J are updated:
//
//   phase 2  row panel (r, J), J > r: D_rJ = min(D_rJ, D_rr (x) D_rJ);
//            column panel (I, r), I < r: D_Ir = min(D_Ir, D_Ir (x) D_rr);
//   phase 3  (I, J), I <= J, I, J != r: D_IJ = min(D_IJ, D_Ir (x) D_rJ).
//
// Phase 3 needs D_Ir for I > r and D_rJ for J < r, blocks below the
// diagonal.  By symmetry both are pieces of block row r: D_Ir[i][k] =
// D_rI[k][i] and D_rJ = D_Jr^T.  So phase 2 writes each panel block it
// produces a second time, into a copy R of block row r (128 x 128q words):
// R[k][x] = D_rx, taken from the row block (r, x) as is for x > r and from
// the column block (x, r) transposed for x < r.  Phase 3 then reads only R:
// D_IJ = min(D_IJ, R_I^T (x) R_J), R_I the 128 columns of block I of R, both
// operands k-major, which is the layout direct-to-LDS staging needs.
//
// Every candidate D_Ik + D_kJ of the full method is formed here from the
// same two values (fp32 addition is commutative), so the result is the
// full method's, bit for bit, at about half its phase-2 and phase-3 work.
// The strict lower triangle is filled from the upper one at the end (and
// once before the first round, so the input's lower triangle is never read).
//
// Rounds overlap as in the full solver: phase 3 of round r is split into the
// tiles in block row/column r+1 (with the closure of diagonal block r+1,
// phase 1 of round r+1, fused), which stay on the caller's stream, and the
// rest, which a helper stream runs while the caller's stream goes on with
// phase 2 of round r+1.  The copies of rounds r and r+1 use two slots.
#include "apsp_tile.h"
#include "apsp_tilemap.h"

namespace apsp {

namespace {

using tile::NT;
using tile::TB;

using tilemap::kSymAll;
using tilemap::kSymNext;
using tilemap::kSymRest;

// Phase 2 of round r: tiles (r, J), J > r, then (I, r), I < r (q-1 of them),
// stored in place and into R (row block as is, column block transposed).
template <class Op>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_sym_panels(
    uint32_t *__restrict__ D, int64_t ld, int64_t n, int r, int q, int vec,
    uint32_t *__restrict__ R, int64_t ldr) {
    __shared__ tile::Lds L;
    tile::chain_priority();
    const int t = blockIdx.x;
    int I, J;
    if (t < q - 1 - r) {
        I = r;
        J = r + 1 + t;
    } else {
        I = t - (q - 1 - r);
        J = r;
    }
    const int64_t i0 = (int64_t)I * TB, j0 = (int64_t)J * TB, kb = (int64_t)r * TB;
    const int kw = (int)((n - kb) < TB ? (n - kb) : TB);
    const int mr = (int)((n - i0) < TB ? (n - i0) : TB);
    const int nc = (int)((n - j0) < TB ? (n - j0) : TB);
    uint32_t acc[8][8];
    tile::load_acc<Op, false>(acc, D, ld, i0, j0, mr, nc, vec);
    tile::minplus_tile<Op, false>(acc, D, ld, i0, j0, kb, mr, nc, kw, vec, L);
    tile::store_acc<Op>(acc, D, ld, i0, j0, mr, nc, vec);
    if (I == r)
        tile::store_acc<Op>(acc, R, ldr, 0, j0, mr, nc, true);  // rows are k (mr == kw)
    else
        tile::store_acc_t<Op>(acc, R, ldr, i0, mr, nc);  // columns are k (nc == kw)
}

// Phase 3 on a tile set from R.  DIRECT: n a multiple of 128 and D's rows
// 16-byte aligned, every tile full; both operands staged straight into LDS.
// Otherwise the register-staged loader reads A transposed from R with the
// tile's bounds.  kSymNext (and kSymAll with `close`) closes diagonal block
// r+1 after its update.
template <class Op, int SET, bool DIRECT>
__device__ __forceinline__ void sym_update(uint32_t *D, int64_t ld, int64_t n, int r, int q,
                                           int vec, const uint32_t *R, int64_t ldr, int close,
                                           tile::Lds &L) {
    int I, J;
    tilemap::sym_tile_of<SET>((int)blockIdx.x, r, q, I, J);
    const int64_t i0 = (int64_t)I * TB, j0 = (int64_t)J * TB, kb = (int64_t)r * TB;
    const int kw = (int)((n - kb) < TB ? (n - kb) : TB);
    const int mr = (int)((n - i0) < TB ? (n - i0) : TB);
    const int nc = (int)((n - j0) < TB ? (n - j0) : TB);
    const bool closes = (SET == kSymNext || close) && I == r + 1 && J == r + 1;
    uint32_t acc[8][8];
    if (DIRECT) {
        tile::io_direct(acc, D + i0 * ld + j0, (uint32_t)ld, false);
        tile::minplus_tile_direct<Op>(acc, R, R, TB, ldr, R, ldr, i0, j0, TB, L);
        if (closes) tile::close_block<Op>(acc, TB, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
        uint32_t *base = D + i0 * ld + j0;
        uint32_t ldu = (uint32_t)ld;
        asm volatile("" : "+s"(base), "+s"(ldu));
        tile::io_direct(acc, base, ldu, true);
    } else {
        tile::load_acc<Op, false>(acc, D, ld, i0, j0, mr, nc, vec);
        tile::minplus_tile_ab<Op, false, true, false>(acc, R, ldr, R, ldr, i0, j0, mr, nc, kw,
                                                      true, L);
        if (closes) tile::close_block<Op>(acc, mr, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
        tile::store_acc<Op>(acc, D, ld, i0, j0, mr, nc, vec);
    }
}

// The bulk set on the helper stream: 4 workgroups per CU in direct form.
template <class Op, bool DIRECT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(DIRECT ? 4 : 3))) void k_sym_rest(
    uint32_t *__restrict__ D, int64_t ld, int64_t n, int r, int q, int vec,
    const uint32_t *__restrict__ R, int64_t ldr) {
    __shared__ tile::Lds L;
    sym_update<Op, kSymRest, DIRECT>(D, ld, n, r, q, vec, R, ldr, 0, L);
}

// The caller-stream sets (kSymNext, kSymAll): they carry the closure.
template <class Op, int SET, bool DIRECT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_sym_chain(
    uint32_t *__restrict__ D, int64_t ld, int64_t n, int r, int q, int vec,
    const uint32_t *__restrict__ R, int64_t ldr, int close) {
    __shared__ tile::Lds L;
    tile::chain_priority();
    sym_update<Op, SET, DIRECT>(D, ld, n, r, q, vec, R, ldr, close, L);
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

unsigned set_size(int set, int q) {
    switch (set) {
    case kSymAll: return (unsigned)((q - 1) * q / 2);
    case kSymRest: return (unsigned)((q - 2) * (q - 1) / 2);
    default: return (unsigned)(q - 1);
    }
}

struct SymLaunch {
    uint32_t *D;
    int64_t ld, n;
    int q, vec, dtype;
    bool direct;

    template <class Op>
    hipError_t panels_t(int r, uint32_t *R, int64_t ldr, hipStream_t s) const {
        hipLaunchKernelGGL((k_sym_panels<Op>), dim3((unsigned)(q - 1)), dim3(NT), 0, s, D, ld, n,
                           r, q, vec, R, ldr);
        return hipGetLastError();
    }
    hipError_t panels(int r, uint32_t *R, int64_t ldr, hipStream_t s) const {
        return dtype == 0 ? panels_t<OpI32>(r, R, ldr, s) : panels_t<OpF32>(r, R, ldr, s);
    }

    template <class Op, bool DIRECT>
    hipError_t update_t(int r, int set, const uint32_t *R, int64_t ldr, int close,
                        hipStream_t s) const {
        const unsigned g = set_size(set, q);
        if (g == 0) return hipSuccess;
        if (set == kSymRest)
            hipLaunchKernelGGL((k_sym_rest<Op, DIRECT>), dim3(g), dim3(NT), 0, s, D, ld, n, r, q,
                               vec, R, ldr);
        else if (set == kSymNext)
            hipLaunchKernelGGL((k_sym_chain<Op, kSymNext, DIRECT>), dim3(g), dim3(NT), 0, s, D,
                               ld, n, r, q, vec, R, ldr, close);
        else
            hipLaunchKernelGGL((k_sym_chain<Op, kSymAll, DIRECT>), dim3(g), dim3(NT), 0, s, D,
                               ld, n, r, q, vec, R, ldr, close);
        return hipGetLastError();
    }
    hipError_t update(int r, int set, const uint32_t *R, int64_t ldr, int close,
                      hipStream_t s) const {
        if (dtype == 0)
            return direct ? update_t<OpI32, true>(r, set, R, ldr, close, s)
                          : update_t<OpI32, false>(r, set, R, ldr, close, s);
        return direct ? update_t<OpF32, true>(r, set, R, ldr, close, s)
                      : update_t<OpF32, false>(r, set, R, ldr, close, s);
    }
};

}  // namespace

hipError_t run_symmetric(uint32_t *D, int64_t n, int64_t ld, int dtype, hipStream_t caller) {
    if (n <= 0) return hipSuccess;
    hipStream_t s = caller;  // the caller's stream, then the state's chain stream
    const int nb = (int)((n + 63) / 64);
    const dim3 mgrid((unsigned)((int64_t)nb * (nb + 1) / 2));
    auto mirror = [&]() {
        hipLaunchKernelGGL(k_mirror, mgrid, dim3(256), 0, s, D, ld, n, nb);
        return hipGetLastError();
    };
    hipError_t e = launch_prologue(D, n, ld, dtype, s);
    // the input's lower triangle is not read: make the matrix symmetric first
    if (e == hipSuccess) e = mirror();
    if (e == hipSuccess) e = launch_phase1(D, n, ld, dtype, 0, s);
    const int q = (int)((n + TB - 1) / TB);
    if (q == 1 || e != hipSuccess) return e == hipSuccess ? mirror() : e;

    SideResources res;
    std::unique_lock<std::mutex> lock;
    e = side_resources(caller, n, &res, &lock);
    if (e != hipSuccess) return e;
    // the rounds run on the chain stream (after the caller's earlier work) and
    // the helper stream, which sit on different hardware queues
    e = hipEventRecord(res.enter, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(res.chain, res.enter, 0);
    if (e != hipSuccess) return e;
    s = res.chain;
    SymLaunch L;
    L.D = D;
    L.ld = ld;
    L.n = n;
    L.q = q;
    L.vec = ((reinterpret_cast<uintptr_t>(D) & 15u) == 0 && (ld & 3) == 0) ? 1 : 0;
    L.dtype = dtype;
    // full tiles, aligned rows, 32-bit lane offsets (128 ld and 128 ldr < 2^30)
    L.direct = n % TB == 0 && L.vec && ld < ((int64_t)1 << 22) && res.ld < ((int64_t)1 << 22);

    if (q == 2) {  // no rest set to overlap: round by round on the chain stream
        for (int r = 0; r < q && e == hipSuccess; ++r) {
            uint32_t *R = res.slot[r & 1];
            e = L.panels(r, R, res.ld, s);
            if (e == hipSuccess) e = L.update(r, kSymAll, R, res.ld, r + 1 < q ? 1 : 0, s);
        }
    } else {
        // round r: phase 2 (phase 1 ran fused in the previous round's next
        // set), then the rest set on the helper stream once phase 2 is done,
        // and the next set on the chain stream after the previous round's
        // rest set (it rewrites tiles in block row/column r+1, which that set
        // wrote); the previous rest set also read the copy slot that phase 2
        // of round r+1 overwrites, which that same wait orders.
        for (int r = 0; r < q && e == hipSuccess; ++r) {
            uint32_t *R = res.slot[r & 1];
            e = L.panels(r, R, res.ld, s);
            if (e == hipSuccess && r > 0) e = hipStreamWaitEvent(s, res.rest_done, 0);
            if (e != hipSuccess) break;
            if (r + 1 < q) {
                e = hipEventRecord(res.p2_done, s);
                if (e == hipSuccess) e = hipStreamWaitEvent(res.side, res.p2_done, 0);
                if (e == hipSuccess) e = L.update(r, kSymRest, R, res.ld, 0, res.side);
                if (e == hipSuccess) e = hipEventRecord(res.rest_done, res.side);
                if (e == hipSuccess) e = L.update(r, kSymNext, R, res.ld, 1, s);
            } else {
                e = L.update(r, kSymAll, R, res.ld, 0, s);
            }
        }
    }
    if (e == hipSuccess) e = mirror();  // blocks below the diagonal were not updated
    // the caller's stream waits for the chain, which waited for the helper
    if (e == hipSuccess) e = hipEventRecord(res.leave, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(caller, res.leave, 0);
    if (e != hipSuccess) note_error("symmetric solve launch", e);
    return e;
}

}  // namespace apsp

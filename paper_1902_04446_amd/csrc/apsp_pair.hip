// Round pairs for the single-graph solver: phase 3 of rounds r and r+1 in one
// pass over each tile (arXiv:1902.04446, Sec. 4.4/4.5: the three phases of
// Algorithms 3 and 4, applied to two consecutive rounds).
//
// For a tile (I, J) outside block rows/columns r and r+1, the two rounds'
// phase-3 updates are
//     D'  = min(D,  D'[I,r] (x) D'[r,J])                 round r
//     D'' = min(D', D''[I,r+1] (x) D''[r+1,J])           round r+1
// where D'[., r] / D'[r, .] are round r's panels (after its phase 2) and
// D''[., r+1] / D''[r+1, .] round r+1's.  Since min is exact and every
// candidate is one addition, D'' = min(D, both products): one pass with k
// over blocks r and r+1 (256 wide) gives the same bits, reading and writing
// the tile once instead of twice.  That needs block column r and block row r
// to hold round r's panels during the pass, so round r+1's phase 3 on those
// tiles (their "pending" update) is deferred:
//   * tiles (x, r), (r, x) for the next pair's blocks x = r+2, r+3 get it
//     right after the next pair's first tiles are done (kFix, next);
//   * the other tiles of block row/column r get it at the start of their
//     update in the next pair's pass, from a copy of round r+1's panels
//     taken when phase 2 of round r+1 wrote them (by then the next pair may
//     have changed block row/column r+1 in the matrix itself; the column
//     panel is copied transposed);
//   * at the end of a call, kFix (final) applies what is left, so a call
//     always leaves exactly the state of Floyd-Warshall after its last round.
// The schedule (apsp_runtime.hip) keeps every read of these tiles ahead of
// every write to them; the result is the same as running the rounds one by
// one, bit for bit.
//
// The rest pass (kRest2, ~98% of the work) has a second form for fp32
// matrices whose tiles are all full and rows 16-byte aligned: the operands go
// from memory straight to LDS (tile::minplus_tile_direct), the column panels
// of rounds r and r+1 read from their transposed copies (phase 2 of each
// round writes one), the row panels from the matrix.  Fewer registers per
// thread let 4 workgroups share a CU instead of 3.  It forms the same
// candidates and minima, so the same bits.
#include <algorithm>

#include "apsp_tile.h"
#include "apsp_tilemap.h"

namespace apsp {

namespace {

using tile::NT;
using tile::TB;

using tilemap::kPanelsSnap;
using tilemap::kNext2;
using tilemap::kRest2;
using tilemap::kFix;
using tilemap::kNextR;
using tilemap::kRest1;

struct PairArgs {
    uint32_t *D;
    int64_t ld, n;
    int r;       // first round of the pair (kPanelsSnap: the panel round)
    int q;
    int vec;     // 16-byte aligned rows of D
    int nxt;     // next-pair blocks present: r+2, r+3 below q (0..2)
    int close;   // kNext2: close diagonal block r+2 after its update
    int lo, hi;  // kRest2: band [lo, hi) of block rows
    int prev;    // kNext2/kRest2: first round of the previous pair, -1 if none
    int final_;  // kFix: 0 = tiles (x, r), (r, x) for next blocks x; 1 = the rest
    const uint32_t *prow;   // copy of the previous pair's round prev+1 block row
    const uint32_t *pcolT;  // ... and its block column, transposed
    const uint32_t *at0;    // kRest2 direct: round r's block column, transposed
    const uint32_t *at1;    // ... and round r+1's
    int64_t ldc;            // leading dimension of the copies
    uint32_t *srow;         // kPanelsSnap: block-row copy to write (or null)
    uint32_t *scolT;        // kPanelsSnap: transposed block-column copy to write
};

__device__ __forceinline__ int width(int64_t n, int blk) {
    const int64_t w = n - (int64_t)blk * TB;
    return (int)(w < TB ? w : TB);
}

// Workgroup -> tile and its update: k blocks [kb, kb + kblocks), deferred
// update first (pending), closure after (close).
struct Job {
    int I, J, kb, kblocks;
    bool pending, close;
};

template <int MODE>
__device__ __forceinline__ Job job_of(const PairArgs &a) {
    Job j{0, 0, a.r, 2, false, false};
    tilemap::pair_tile_of<MODE>((int)blockIdx.x, a.r, a.q, a.nxt, a.lo, a.hi, a.final_, j.I, j.J);
    const int r = a.r;
    if (MODE == kPanelsSnap) {
        j.kb = r;
        j.kblocks = 1;
        return j;
    }
    if (MODE == kFix) {
        j.kb = r + 1;
        j.kblocks = 1;
        return j;
    }
    if (MODE == kRest1) {
        j.kblocks = 1;
        return j;
    }
    if (MODE == kNextR) {
        j.kblocks = 1;
        j.close = a.close && j.I == r + 1 && j.J == r + 1;
        return j;
    }
    if (MODE == kNext2) j.close = a.close && j.I == r + 2 && j.J == r + 2;
    j.pending = a.prev >= 0 && (j.I == a.prev || j.J == a.prev) && j.I != a.prev + 1 &&
                j.J != a.prev + 1;
    return j;
}

template <class Op, int MODE, bool NORM>
__device__ __forceinline__ void pair_update(const PairArgs &a, tile::Lds &L) {
    const Job jb = job_of<MODE>(a);
    const int64_t i0 = (int64_t)jb.I * TB, j0 = (int64_t)jb.J * TB;
    const int mr = width(a.n, jb.I), nc = width(a.n, jb.J);
    const int64_t kb = (int64_t)jb.kb * TB;
    const int64_t kwl = a.n - kb;
    const int kw = (int)(kwl < (int64_t)jb.kblocks * TB ? kwl : (int64_t)jb.kblocks * TB);
    const bool vec = a.vec != 0;

    // the rest set's tiles are each read and written once per pair: stream them
    constexpr bool kStream = MODE == kRest2;
    uint32_t acc[8][8];
    tile::load_acc<Op, NORM, kStream>(acc, a.D, a.ld, i0, j0, mr, nc, vec);
    if (MODE != kPanelsSnap && MODE != kFix && jb.pending)
        // round prev+1 on a tile of block row/column prev, from the copies
        // (the column panel's is transposed)
        tile::minplus_tile_ab<Op, NORM, true, false>(acc, a.pcolT, a.ldc, a.prow, a.ldc, i0, j0,
                                                     mr, nc, width(a.n, a.prev + 1), true, L);
    tile::minplus_tile<Op, NORM>(acc, a.D, a.ld, i0, j0, kb, mr, nc, kw, vec, L);
    if (MODE == kNext2 && jb.close)  // phase 1 of round r+2, fused
        tile::close_block<Op>(acc, mr, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
    tile::store_acc<Op, kStream>(acc, a.D, a.ld, i0, j0, mr, nc, vec);
    if (MODE == kPanelsSnap) {
        if (jb.I == a.r) {  // block row: row k of the copy holds row k of the block
            if (a.srow) tile::store_acc<Op>(acc, a.srow, a.ldc, 0, j0, mr, nc, true);
        } else {            // block column: column k of the block at row k of the copy
            tile::store_acc_t<Op>(acc, a.scolT, a.ldc, i0, mr, nc);
        }
    }
}

// The rest pass of a pair with direct staging (full tiles of an aligned fp32
// matrix): the column panels from their transposed copies, the row panels
// from the matrix; the output tile through tile::io_direct.
template <class Op, int MODE>
__device__ __forceinline__ void pair_direct_update(const PairArgs &a, tile::Lds &L) {
    const Job jb = job_of<MODE>(a);
    const int64_t i0 = (int64_t)jb.I * TB, j0 = (int64_t)jb.J * TB;
    uint32_t acc[8][8];
    tile::io_direct(acc, a.D + i0 * a.ld + j0, (uint32_t)a.ld, false);
    // product 0: round prev+1's deferred update from the copies (pending
    // tiles only); product 1: rounds r and r+1.  One call site keeps the
    // register count at 4 workgroups per CU.
#pragma unroll 1
    for (int x = jb.pending ? 0 : 1; x < 2; ++x) {
        const uint32_t *at0 = x ? a.at0 : a.pcolT, *at1 = x ? a.at1 : a.pcolT;
        const uint32_t *B = x ? a.D + (int64_t)a.r * TB * a.ld : a.prow;
        tile::minplus_tile_direct<Op>(acc, at0, at1, TB, a.ldc, B, x ? a.ld : a.ldc, i0, j0,
                                         x ? jb.kblocks * TB : TB, L);
    }
    if (MODE != kRest2 && jb.close)  // phase 1 of round r+2 (kNext2) or r+1 (kNextR), fused
        tile::close_block<Op>(acc, TB, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
    uint32_t *base = a.D + i0 * a.ld + j0;
    uint32_t ld = (uint32_t)a.ld;
    asm volatile("" : "+s"(base), "+s"(ld));
    tile::io_direct(acc, base, ld, true);
}

template <class Op, int MODE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_pair(PairArgs a) {
    __shared__ tile::Lds L;
    if (MODE != kRest2) tile::chain_priority();
    pair_update<Op, MODE, false>(a, L);
}

// The rest pass (kRest2) and the pass on block rows/columns r+2, r+3
// (kNext2, with its closure) in direct-staged form.  The chain launches
// (kNext2 among them) run beside the previous pair's bands, whose workgroups
// fill a CU 4 at a time with 120 registers each (480 of 512 per SIMD): a
// chain workgroup gets a CU as soon as one band workgroup ends only if it
// needs at most 152, which the other chain kernels do (138-144) but the
// register-staged kNext2 (154) does not.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_pair_rest_direct(
    PairArgs a) {
    __shared__ tile::Lds L;
    pair_direct_update<OpF32, kRest2>(a, L);
}

// A single round's rest set (kRest1) in the same direct form, for matrices
// solved in single rounds: the column panel from its transposed copy.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_round_rest_direct(
    PairArgs a) {
    __shared__ tile::Lds L;
    pair_direct_update<OpF32, kRest1>(a, L);
}

// kNext2 and kNextR (with the closure's registers: at most 152, 3 workgroups
// per CU)
template <int MODE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_pair_next_direct(
    PairArgs a) {
    __shared__ tile::Lds L;
    tile::chain_priority();
    pair_direct_update<OpF32, MODE>(a, L);
}

// The same direct-staged kernels for an int32 matrix held as kI32AsF32:
// fp32 arithmetic on its fp32 bits when *wmax allows it (IF_EXACT, Op =
// OpF32), uint32 arithmetic on the untouched words otherwise (Op = OpI32);
// neither converts anything, so both stage straight into LDS.  Each pass is
// launched as both kernels, and the one whose case does not hold returns at
// once: one kernel holding both cases measured 123 and 155 VGPRs against the
// 120 and 152 that keep the bands at 4 workgroups per CU and the chain's
// workgroups able to start beside them.
template <class Op, bool IF_EXACT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_pair_rest_direct_i32(
    PairArgs a, const uint32_t *__restrict__ wmax) {
    if (int_exact_in_f32(a.n, *wmax) != IF_EXACT) return;
    __shared__ tile::Lds L;
    pair_direct_update<Op, kRest2>(a, L);
}

template <class Op, bool IF_EXACT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_round_rest_direct_i32(
    PairArgs a, const uint32_t *__restrict__ wmax) {
    if (int_exact_in_f32(a.n, *wmax) != IF_EXACT) return;
    __shared__ tile::Lds L;
    pair_direct_update<Op, kRest1>(a, L);
}

template <int MODE, class Op, bool IF_EXACT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_pair_next_direct_i32(
    PairArgs a, const uint32_t *__restrict__ wmax) {
    if (int_exact_in_f32(a.n, *wmax) != IF_EXACT) return;
    __shared__ tile::Lds L;
    tile::chain_priority();
    pair_direct_update<Op, MODE>(a, L);
}

// int32 on the fp32 pipe (OpI32F, bit-identical) when *wmax allows it; CONV:
// the matrix is held as kI32AsF32, so that case computes as OpF32 with no
// conversion.
template <int MODE, bool CONV>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_pair_i32(
    PairArgs a, const uint32_t *__restrict__ wmax) {
    __shared__ tile::Lds L;
    if (MODE != kRest2) tile::chain_priority();
    if (int_exact_in_f32(a.n, *wmax)) {
        if (CONV)
            pair_update<OpF32, MODE, false>(a, L);
        else
            pair_update<OpI32F, MODE, true>(a, L);
    } else {
        pair_update<OpI32, MODE, false>(a, L);
    }
}

template <int MODE>
hipError_t launch(const PairArgs &a, int dtype, const uint32_t *wmax, unsigned grid,
                  hipStream_t s) {
    if (grid == 0) return hipSuccess;
    if (dtype == kI32AsF32)
        hipLaunchKernelGGL((k_pair_i32<MODE, true>), dim3(grid), dim3(NT), 0, s, a, wmax);
    else if (dtype == 0 && wmax)
        hipLaunchKernelGGL((k_pair_i32<MODE, false>), dim3(grid), dim3(NT), 0, s, a, wmax);
    else if (dtype == 0)
        hipLaunchKernelGGL((k_pair<OpI32, MODE>), dim3(grid), dim3(NT), 0, s, a);
    else
        hipLaunchKernelGGL((k_pair<OpF32, MODE>), dim3(grid), dim3(NT), 0, s, a);
    return hipGetLastError();
}

PairArgs base_args(uint32_t *D, int64_t n, int64_t ld, int r, const PairCopies &c) {
    PairArgs a{};
    a.D = D;
    a.ld = ld;
    a.n = n;
    a.r = r;
    a.q = (int)num_rounds(n);
    a.vec = ((reinterpret_cast<uintptr_t>(D) & 15u) == 0 && (ld & 3) == 0) ? 1 : 0;
    const int nx = a.q - (r + 2);
    a.nxt = nx < 0 ? 0 : (nx > 2 ? 2 : nx);
    a.prev = -1;
    a.ldc = c.ld;
    return a;
}

}  // namespace

int pair_next_blocks(int64_t n, int64_t r) {
    const int64_t nx = num_rounds(n) - (r + 2);
    return (int)(nx < 0 ? 0 : (nx > 2 ? 2 : nx));
}

int64_t pair_rest_count(int64_t n, int64_t r, int64_t lo, int64_t hi) {
    const int64_t q = num_rounds(n);
    if (r < 0 || r + 1 >= q || lo >= hi) return 0;
    const int64_t e1 = r + 2 + pair_next_blocks(n, r);
    const int64_t x0 = std::max(r, lo), x1 = std::min(e1, hi);
    const int64_t rows = hi - lo - (x1 > x0 ? x1 - x0 : 0);
    return rows > 0 ? rows * (q - (e1 - r)) : 0;
}

bool pair_rest_direct(const uint32_t *D, int64_t n, int64_t ld, int dtype) {
    return (dtype == 1 || dtype == kI32AsF32) && n % TB == 0 && (reinterpret_cast<uintptr_t>(D) & 15u) == 0 &&
           (ld & 3) == 0 && ld < ((int64_t)1 << 23);
}

hipError_t launch_pair_panels(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t pr,
                              const PairCopies &c, int row_slot, int col_slot, hipStream_t s,
                              const uint32_t *wmax) {
    PairArgs a = base_args(D, n, ld, (int)pr, c);
    a.srow = row_slot >= 0 ? c.row[row_slot] : nullptr;
    a.scolT = c.colT[col_slot];
    return launch<kPanelsSnap>(a, dtype, wmax, (unsigned)(2 * (a.q - 1)), s);
}

hipError_t launch_pair_next(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                            bool close, int64_t prev, const PairCopies &c, int prev_slot,
                            int first_slot, int slot, hipStream_t s, const uint32_t *wmax) {
    PairArgs a = base_args(D, n, ld, (int)r, c);
    a.close = close ? 1 : 0;
    a.prev = (int)prev;
    if (prev >= 0) {
        a.prow = c.row[prev_slot];
        a.pcolT = c.colT[prev_slot];
    }
    const int m = a.q - 2;
    const unsigned count = (unsigned)(a.nxt * m + a.nxt * (m - a.nxt));
    if (count > 0 && pair_rest_direct(D, n, ld, dtype)) {
        a.at0 = c.colT[first_slot];
        a.at1 = c.colT[slot];
        if (dtype == kI32AsF32) {
            hipLaunchKernelGGL((k_pair_next_direct_i32<kNext2, OpF32, true>), dim3(count),
                               dim3(NT), 0, s, a, wmax);
            hipLaunchKernelGGL((k_pair_next_direct_i32<kNext2, OpI32, false>), dim3(count),
                               dim3(NT), 0, s, a, wmax);
        } else
            hipLaunchKernelGGL(k_pair_next_direct<kNext2>, dim3(count), dim3(NT), 0, s, a);
        return hipGetLastError();
    }
    return launch<kNext2>(a, dtype, wmax, count, s);
}

hipError_t launch_pair_round_next(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                                  const PairCopies &c, int first_slot, hipStream_t s,
                                  const uint32_t *wmax) {
    if (!pair_rest_direct(D, n, ld, dtype))
        return launch_tile_set(D, n, ld, dtype, r, kNext, s, true, wmax);
    PairArgs a = base_args(D, n, ld, (int)r, c);
    if (r + 1 >= a.q) return hipSuccess;
    a.close = 1;
    a.at0 = c.colT[first_slot];
    a.at1 = a.at0;
    if (dtype == kI32AsF32) {
        hipLaunchKernelGGL((k_pair_next_direct_i32<kNextR, OpF32, true>),
                           dim3((unsigned)(2 * a.q - 3)), dim3(NT), 0, s, a, wmax);
        hipLaunchKernelGGL((k_pair_next_direct_i32<kNextR, OpI32, false>),
                           dim3((unsigned)(2 * a.q - 3)), dim3(NT), 0, s, a, wmax);
    } else
        hipLaunchKernelGGL(k_pair_next_direct<kNextR>, dim3((unsigned)(2 * a.q - 3)), dim3(NT), 0,
                           s, a);
    return hipGetLastError();
}

hipError_t launch_pair_rest(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                            int64_t lo, int64_t hi, int64_t prev, const PairCopies &c,
                            int prev_slot, int first_slot, int slot, hipStream_t s,
                            const uint32_t *wmax) {
    const int64_t count = pair_rest_count(n, r, lo, hi);
    if (count <= 0) return hipSuccess;
    PairArgs a = base_args(D, n, ld, (int)r, c);
    a.lo = (int)lo;
    a.hi = (int)hi;
    a.prev = (int)prev;
    if (prev >= 0) {
        a.prow = c.row[prev_slot];
        a.pcolT = c.colT[prev_slot];
    }
    if (pair_rest_direct(D, n, ld, dtype)) {
        a.at0 = c.colT[first_slot];
        a.at1 = c.colT[slot];
        if (dtype == kI32AsF32) {
            hipLaunchKernelGGL((k_pair_rest_direct_i32<OpF32, true>), dim3((unsigned)count),
                               dim3(NT), 0, s, a, wmax);
            hipLaunchKernelGGL((k_pair_rest_direct_i32<OpI32, false>), dim3((unsigned)count),
                               dim3(NT), 0, s, a, wmax);
        } else
            hipLaunchKernelGGL(k_pair_rest_direct, dim3((unsigned)count), dim3(NT), 0, s, a);
        return hipGetLastError();
    }
    return launch<kRest2>(a, dtype, wmax, (unsigned)count, s);
}

hipError_t launch_round_rest_direct(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                                   int64_t lo, int64_t hi, const PairCopies &c, int col_slot,
                                   hipStream_t s, const uint32_t *wmax) {
    const int64_t count = tilemap::tile_count(num_rounds(n), r, kRest, lo, hi);
    if (count <= 0) return hipSuccess;
    PairArgs a = base_args(D, n, ld, (int)r, c);
    a.lo = (int)lo;
    a.hi = (int)hi;
    a.at0 = c.colT[col_slot];
    a.at1 = a.at0;
    if (dtype == kI32AsF32) {
        hipLaunchKernelGGL((k_round_rest_direct_i32<OpF32, true>), dim3((unsigned)count), dim3(NT),
                           0, s, a, wmax);
        hipLaunchKernelGGL((k_round_rest_direct_i32<OpI32, false>), dim3((unsigned)count),
                           dim3(NT), 0, s, a, wmax);
    } else
        hipLaunchKernelGGL(k_round_rest_direct, dim3((unsigned)count), dim3(NT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pair_fix(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                           bool final_, hipStream_t s, const uint32_t *wmax) {
    PairArgs a = base_args(D, n, ld, (int)r, PairCopies{});
    a.final_ = final_ ? 1 : 0;
    const unsigned count = final_ ? (unsigned)((a.q - 1 - a.nxt) + (a.q - 2 - a.nxt))
                                  : (unsigned)(2 * a.nxt);
    return launch<kFix>(a, dtype, wmax, count, s);
}

}  // namespace apsp

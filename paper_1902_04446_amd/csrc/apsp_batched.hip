// Many independent graphs (the blocked method of arXiv:1902.04446, Sec.
// 4.4/4.5, Algorithms 3 and 4, applied to each graph), solved together.
//
// Round-synchronous batching: every launch covers one phase of one round for
// all graphs that have that round, one workgroup per 128 x 128 tile, with
// the same register-blocked min-plus update as the single-graph solver
// (tile::minplus_tile).  The tiles of one graph spread over many CUs, so a
// large graph is not bound to the speed of one CU, and every workgroup does
// the same amount of work, so no longest-job-first ordering is needed.
//
//   launch 0          phase 1 of round 0 for every graph (closure of its
//                     first diagonal block; a graph with n <= 128 is done);
//   launch 2r+1       phase 2 of round r (block row and column r);
//   launch 2r+2       phase 3 of round r; the workgroup of diagonal block
//                     r+1 also closes it (phase 1 of round r+1) before
//                     storing it, so no separate phase-1 launch is needed.
//
// The work items (graph, I, J) of a launch are grouped per XCD: a graph's
// tiles all go to the XCD g % 8 (workgroup w runs on XCD w % 8), so the
// panel blocks a graph's tiles share stay in one L2.  The input
// normalisation (zero diagonal, int32 clamp at 2^30) is applied as tiles
// are loaded; it is idempotent.
#include "apsp_tile.h"

namespace apsp {

namespace {

using tile::NT;
using tile::TB;

template <class Op, bool CLOSE_ONLY>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_batched(
    const BatchDesc *__restrict__ descs, const BatchItem *__restrict__ items, XcdRanges ranges,
    int r) {
    __shared__ tile::Lds L;
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    if (slot >= ranges.count[x]) return;  // this XCD's list is shorter
    const BatchItem it = items[ranges.offset[x] + slot];
    const BatchDesc g = descs[it.graph];
    uint32_t *D = g.ptr;
    const int n = g.n;
    const int64_t ld = g.ld;
    const bool vec = ((reinterpret_cast<uintptr_t>(D) & 15u) == 0) && ((ld & 3) == 0);
    const int I = it.ij >> 16, J = it.ij & 0xffff;
    const int64_t kb = (int64_t)r * TB, i0 = (int64_t)I * TB, j0 = (int64_t)J * TB;
    const int kw = (n - (int)kb) < TB ? (n - (int)kb) : TB;
    const int mr = (n - (int)i0) < TB ? (n - (int)i0) : TB;
    const int nc = (n - (int)j0) < TB ? (n - (int)j0) : TB;

    uint32_t acc[8][8];
    tile::load_acc<Op, true>(acc, D, ld, i0, j0, mr, nc, vec);
    if (CLOSE_ONLY) {
        tile::close_block<Op>(acc, kw, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
    } else {
        tile::minplus_tile<Op, true>(acc, D, ld, i0, j0, kb, mr, nc, kw, vec, L);
        if (I == r + 1 && J == r + 1)  // phase 1 of round r+1, fused
            tile::close_block<Op>(acc, mr, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
    }
    tile::store_acc<Op>(acc, D, ld, i0, j0, mr, nc, vec);
}

}  // namespace


hipError_t launch_batched_items(const BatchDesc *descs, const BatchItem *items,
                                const XcdRanges &ranges, int r, bool close_only, int dtype,
                                hipStream_t s) {
    int longest = 0;
    for (int x = 0; x < 8; ++x) longest = ranges.count[x] > longest ? ranges.count[x] : longest;
    if (longest == 0) return hipSuccess;
    const dim3 grid((unsigned)longest * 8u);
    if (dtype == 0) {
        if (close_only)
            hipLaunchKernelGGL((k_batched<OpI32, true>), grid, dim3(NT), 0, s, descs, items, ranges, r);
        else
            hipLaunchKernelGGL((k_batched<OpI32, false>), grid, dim3(NT), 0, s, descs, items, ranges, r);
    } else {
        if (close_only)
            hipLaunchKernelGGL((k_batched<OpF32, true>), grid, dim3(NT), 0, s, descs, items, ranges, r);
        else
            hipLaunchKernelGGL((k_batched<OpF32, false>), grid, dim3(NT), 0, s, descs, items, ranges, r);
    }
    return hipGetLastError();
}

}  // namespace apsp

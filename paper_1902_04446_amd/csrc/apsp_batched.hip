// Many independent graphs (the blocked method of arXiv:1902.04446, Sec.
// 4.4/4.5, Algorithms 3 and 4, applied to each graph), solved together.
//
// Round-synchronous batching: every launch covers one phase of one round for
// all graphs that have that round, one workgroup per tile.  Each graph has
// its own round width: 128 (the register-blocked min-plus update of the
// single-graph solver, tile::minplus_tile) or 64 (tile64), chosen per size
// bucket by the batched tuning table; graphs of both widths share launches
// (round r of each at its own width).  The tiles of one graph spread over many CUs, so a
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
// The work items (graph, I, J) of a launch are grouped per XCD: all tiles of
// a graph go to one XCD (workgroup w runs on XCD w % 8), so the panel blocks
// a graph's tiles share stay in one L2.  The input normalisation (zero
// diagonal, int32 clamp at 2^30) is applied as tiles are loaded; it is
// idempotent.
//
// int32 graphs: a scan launch first records each graph's largest finite
// weight; a graph with 2 (n-1) wmax < 2^24 then runs on the fp32 pipe
// (OpI32F, bit-identical to uint32 arithmetic for it), any other in uint32.
#include "apsp_tile.h"
#include "apsp_tile64.h"

namespace apsp {

namespace {

using tile::NT;
using tile::TB;

template <class Op, bool CLOSE_ONLY>
__device__ __forceinline__ void batched_item(uint32_t *D, int n, int64_t ld, bool vec, int I, int J,
                                             int r, tile::Lds &L) {
    const int64_t kb = (int64_t)r * TB, i0 = (int64_t)I * TB, j0 = (int64_t)J * TB;
    const int kw = (n - (int)kb) < TB ? (n - (int)kb) : TB;
    const int mr = (n - (int)i0) < TB ? (n - (int)i0) : TB;
    const int nc = (n - (int)j0) < TB ? (n - (int)j0) : TB;

    uint32_t acc[8][8];
    tile::load_acc<Op, true>(acc, D, ld, i0, j0, mr, nc, vec);
    if (CLOSE_ONLY) {
        tile::close_block<Op>(acc, kw, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
    } else {
        // a tile whose valid rows / columns fit in 64 updates only those
        tile::minplus_tile<Op, true, true>(acc, D, ld, i0, j0, kb, mr, nc, kw, vec, L);
        if (I == r + 1 && J == r + 1)  // phase 1 of round r+1, fused
            tile::close_block<Op>(acc, mr, reinterpret_cast<uint32_t *>(&L.As[0][0][0]));
    }
    tile::store_acc<Op>(acc, D, ld, i0, j0, mr, nc, vec);
}

template <class Op, bool CLOSE_ONLY>
__device__ __forceinline__ void batched_item64(uint32_t *D, int n, int64_t ld, bool vec, int I,
                                               int J, int r, tile64::Lds64 &L) {
    using tile64::T64;
    const int kb = r * T64, i0 = I * T64, j0 = J * T64;
    const int kw = (n - kb) < T64 ? (n - kb) : T64;
    const int mr = (n - i0) < T64 ? (n - i0) : T64;
    const int nc = (n - j0) < T64 ? (n - j0) : T64;
    uint32_t acc[4][4];
    tile64::load64<Op>(acc, D, ld, i0, j0, mr, nc, vec);
    if (CLOSE_ONLY) {
        tile64::close64<Op>(acc, kw, L);
    } else {
        tile64::update64<Op>(acc, D, ld, i0, j0, kb, mr, nc, kw, vec, L);
        if (I == r + 1 && J == r + 1)  // phase 1 of round r+1, fused
            tile64::close64<Op>(acc, mr, L);
    }
    tile64::store64<Op>(acc, D, ld, i0, j0, mr, nc, vec);
}

template <class Op, bool CLOSE_ONLY>
__device__ __forceinline__ void any_item(const BatchDesc &g, bool vec, int I, int J, int r,
                                         void *lds) {
    if (g.tile == 64)
        batched_item64<Op, CLOSE_ONLY>(g.ptr, g.n, g.ld, vec, I, J, r,
                                       *reinterpret_cast<tile64::Lds64 *>(lds));
    else
        batched_item<Op, CLOSE_ONLY>(g.ptr, g.n, g.ld, vec, I, J, r,
                                     *reinterpret_cast<tile::Lds *>(lds));
}

// One work item per workgroup: a tile of round r of one graph, at that
// graph's round width (g.tile, 64 or 128).  DT 0: int32 graphs, each on the
// fp32 pipe (OpI32F) when its largest finite weight wmax[graph] allows it
// bit-exactly, else in uint32; DT 1: fp32.  A closure-only launch (phase 1
// of the first round) is bound by its serial pivot chains, so it is built
// for 4 workgroups per CU rather than 3: more closures overlap per CU.  The
// closures take one pivot per barrier here: measured on the 4096-graph
// batch, the pivot-pair form (which needs 3 workgroups per CU to hold its
// two published rows and columns without spilling) was 1.5-2 % slower.
template <int DT, bool CLOSE_ONLY>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(CLOSE_ONLY ? 4 : 3))) void k_batched(
    const BatchDesc *__restrict__ descs, const BatchItem *__restrict__ items, XcdRanges ranges,
    int r, const uint32_t *__restrict__ wmax) {
    constexpr size_t kLds =
        sizeof(tile::Lds) > sizeof(tile64::Lds64) ? sizeof(tile::Lds) : sizeof(tile64::Lds64);
    __shared__ uint4 lds[kLds / sizeof(uint4)];
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    if (slot >= ranges.count[x]) return;  // this XCD's list is shorter
    const BatchItem it = items[ranges.offset[x] + slot];
    const BatchDesc g = descs[it.graph];
    const bool vec = ((reinterpret_cast<uintptr_t>(g.ptr) & 15u) == 0) && ((g.ld & 3) == 0);
    const int I = it.ij >> 16, J = it.ij & 0xffff;
    if (DT == 1)
        any_item<OpF32, CLOSE_ONLY>(g, vec, I, J, r, lds);
    else if (int_exact_in_f32(g.n, wmax[it.graph]))
        any_item<OpI32F, CLOSE_ONLY>(g, vec, I, J, r, lds);
    else
        any_item<OpI32, CLOSE_ONLY>(g, vec, I, J, r, lds);
}

__global__ void k_fill_words(uint32_t *p, int32_t count, uint32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

// wmax[graph] = max(wmax[graph], largest finite (< 2^30) off-diagonal entry
// of the item's 128 x 128 tile).  Each wave reads two tile rows per step, 16
// bytes per lane (coalesced 512-byte row segments); a thread's 16 rows are
// loaded before any is reduced, so they are all in flight at once.
__global__ __launch_bounds__(NT) void k_batched_wmax(const BatchDesc *__restrict__ descs,
                                                     const BatchItem *__restrict__ items,
                                                     XcdRanges ranges, uint32_t *wmax) {
    const int x = blockIdx.x & 7, slot = blockIdx.x >> 3;
    if (slot >= ranges.count[x]) return;
    const BatchItem it = items[ranges.offset[x] + slot];
    const BatchDesc g = descs[it.graph];
    const bool vec = ((reinterpret_cast<uintptr_t>(g.ptr) & 15u) == 0) && ((g.ld & 3) == 0);
    const int I = it.ij >> 16, J = it.ij & 0xffff;
    const int t = threadIdx.x;
    const int c = J * TB + (t & 31) * 4;  // first of this lane's 4 columns
    constexpr int kSteps = TB / (NT / 32);  // 16 rows per thread
    uint4 v[kSteps];
#pragma unroll
    for (int u = 0; u < kSteps; ++u) {
        const int row = I * TB + (t >> 5) + u * (NT / 32);
        v[u] = make_uint4(0u, 0u, 0u, 0u);
        if (row < g.n) {
            const uint32_t *src = g.ptr + (int64_t)row * g.ld;
            if (vec && c + 4 <= g.n) {
                v[u] = *reinterpret_cast<const uint4 *>(src + c);
            } else {
                v[u].x = c + 0 < g.n ? src[c + 0] : 0u;
                v[u].y = c + 1 < g.n ? src[c + 1] : 0u;
                v[u].z = c + 2 < g.n ? src[c + 2] : 0u;
                v[u].w = c + 3 < g.n ? src[c + 3] : 0u;
            }
        }
    }
    uint32_t m = 0;
#pragma unroll
    for (int u = 0; u < kSteps; ++u) {
        const int row = I * TB + (t >> 5) + u * (NT / 32);
        const uint32_t e4[4] = {v[u].x, v[u].y, v[u].z, v[u].w};
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (e4[e] < kInfI32 && c + e != row && e4[e] > m) m = e4[e];
    }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)m, off);
        m = o > m ? o : m;
    }
    if ((t & 63) == 0 && m > 0) atomicMax(&wmax[it.graph], m);
}

}  // namespace

hipError_t launch_batched_wmax(const BatchDesc *descs, const BatchItem *items,
                               const XcdRanges &ranges, uint32_t *wmax, int32_t graphs,
                               hipStream_t s) {
    if (graphs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_words, dim3((graphs + 255) / 256), dim3(256), 0, s, wmax, graphs, 0u);
    int longest = 0;
    for (int x = 0; x < 8; ++x) longest = ranges.count[x] > longest ? ranges.count[x] : longest;
    if (longest > 0)
        hipLaunchKernelGGL(k_batched_wmax, dim3((unsigned)longest * 8u), dim3(NT), 0, s, descs,
                           items, ranges, wmax);
    return hipGetLastError();
}

hipError_t launch_batched_items(const BatchDesc *descs, const BatchItem *items,
                                const XcdRanges &ranges, int r, bool close_only, int dtype,
                                const uint32_t *wmax, hipStream_t s) {
    int longest = 0;
    for (int x = 0; x < 8; ++x) longest = ranges.count[x] > longest ? ranges.count[x] : longest;
    if (longest == 0) return hipSuccess;
    const dim3 grid((unsigned)longest * 8u);
    if (dtype == 0) {
        if (close_only)
            hipLaunchKernelGGL((k_batched<0, true>), grid, dim3(NT), 0, s, descs, items, ranges, r, wmax);
        else
            hipLaunchKernelGGL((k_batched<0, false>), grid, dim3(NT), 0, s, descs, items, ranges, r, wmax);
    } else {
        if (close_only)
            hipLaunchKernelGGL((k_batched<1, true>), grid, dim3(NT), 0, s, descs, items, ranges, r, wmax);
        else
            hipLaunchKernelGGL((k_batched<1, false>), grid, dim3(NT), 0, s, descs, items, ranges, r, wmax);
    }
    return hipGetLastError();
}

}  // namespace apsp

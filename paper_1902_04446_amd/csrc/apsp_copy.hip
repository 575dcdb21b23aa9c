// Working copies of a matrix for the solve entry points: an aligned (and
// possibly larger) copy to run on, and the copy back.  Plain row copies,
// bound by HBM bandwidth.
#include "apsp_common.h"

namespace apsp {

namespace {

// dst[i * ldd + j] = src[i * lds + j] for i, j < n: a working copy's result
// copied back into the caller's matrix.  One workgroup per row at a time;
// each thread moves four words of the row per step, all four loaded before
// any is stored.
__global__ __launch_bounds__(256) void k_copy_rows(uint32_t *__restrict__ dst, int64_t ldd,
                                                   const uint32_t *__restrict__ src, int64_t lds,
                                                   int64_t n) {
    for (int64_t i = blockIdx.x; i < n; i += gridDim.x) {
        const uint32_t *srow = src + i * lds;
        uint32_t *drow = dst + i * ldd;
        for (int64_t c = threadIdx.x; c < n; c += 1024) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = c + 256 * u < n ? srow[c + 256 * u] : 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c + 256 * u < n) drow[c + 256 * u] = v[u];
        }
    }
}

// The nd x nd working copy of an n x n matrix (nd >= n): the matrix, then
// vertices n .. nd-1 with no edges (`none` off the diagonal, 0 on it).
__global__ __launch_bounds__(256) void k_copy_pad(uint32_t *__restrict__ dst, int64_t ldd,
                                                  int64_t nd, const uint32_t *__restrict__ src,
                                                  int64_t lds, int64_t n, uint32_t none) {
    for (int64_t i = blockIdx.x; i < nd; i += gridDim.x) {
        const uint32_t *srow = src + (i < n ? i : 0) * lds;  // read only for i < n
        uint32_t *drow = dst + i * ldd;
        for (int64_t c = threadIdx.x; c < nd; c += 1024) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t j = c + 256 * u;
                v[u] = (i < n && j < n) ? srow[j] : (i == j ? 0u : none);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (c + 256 * u < nd) drow[c + 256 * u] = v[u];
        }
    }
}

// Each workgroup copies one contiguous range of the launch's rows, each of
// its four waves one row at a time (the lanes 64 words apart, four loads in
// flight before the stores).  The graph of the range's first row is found by
// a binary search over row0; later rows step to the next entry as they pass
// its row0.
__global__ __launch_bounds__(256) void k_batch_copy(const BatchCopy *__restrict__ copies,
                                                    int32_t count, int64_t rows, int64_t per,
                                                    int back) {
    const int64_t first = (int64_t)blockIdx.x * per;
    const int64_t last = first + per < rows ? first + per : rows;
    if (first >= last) return;
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (copies[mid].row0 <= first) lo = mid;
        else hi = mid - 1;
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int c = lo;
    for (int64_t row = first + w; row < last; row += 4) {
        while (c + 1 < count && copies[c + 1].row0 <= row) ++c;
        const BatchCopy e = copies[c];
        const int64_t i = row - e.row0;
        const uint32_t *src = back ? e.work + i * e.ld_work : e.user + i * e.ld_user;
        uint32_t *dst = back ? e.user + i * e.ld_user : e.work + i * e.ld_work;
        for (int j = lane; j < e.n; j += 256) {
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = j + 64 * u < e.n ? src[j + 64 * u] : 0u;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (j + 64 * u < e.n) dst[j + 64 * u] = v[u];
        }
    }
}

}  // namespace

hipError_t launch_batch_copies(const BatchCopy *copies, int32_t count, int64_t rows, bool back,
                               hipStream_t s) {
    if (count <= 0 || rows <= 0) return hipSuccess;
    // 16 rows per workgroup (4 per wave), at most 65536 workgroups
    int64_t per = 16;
    if ((rows + per - 1) / per > 65536) per = (rows + 65535) / 65536;
    const unsigned grid = (unsigned)((rows + per - 1) / per);
    hipLaunchKernelGGL(k_batch_copy, dim3(grid), dim3(256), 0, s, copies, count, rows, per,
                       back ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_copy_pad(uint32_t *dst, int64_t ldd, int64_t nd, const uint32_t *src,
                           int64_t lds, int64_t n, uint32_t none, hipStream_t s) {
    if (nd <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(nd < 8192 ? nd : 8192);
    hipLaunchKernelGGL(k_copy_pad, dim3(grid), dim3(256), 0, s, dst, ldd, nd, src, lds, n, none);
    return hipGetLastError();
}

hipError_t launch_copy_rows(uint32_t *dst, int64_t ldd, const uint32_t *src, int64_t lds, int64_t n,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned grid = (unsigned)(n < 8192 ? n : 8192);
    hipLaunchKernelGGL(k_copy_rows, dim3(grid), dim3(256), 0, s, dst, ldd, src, lds, n);
    return hipGetLastError();
}

}  // namespace apsp

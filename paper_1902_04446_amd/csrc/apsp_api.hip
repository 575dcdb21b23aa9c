// C ABI of the APSP library (declared in include/apsp.h).  Arguments are
// checked on the host before any HIP call; kernels are enqueued on the
// caller's stream; nothing here blocks except apsp_validate.
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <utility>
#include <vector>

#include "../../include/apsp.h"
#include "apsp_common.h"


namespace apsp {

namespace {
thread_local char g_last_error[256] = "";
}  // namespace

void note_error(const char *what, hipError_t e) {
    snprintf(g_last_error, sizeof(g_last_error), "%s: %s (%d)", what, hipGetErrorName(e), (int)e);
}

void note_message(const char *what) { snprintf(g_last_error, sizeof(g_last_error), "%s", what); }

}  // namespace apsp

namespace {

constexpr int64_t kMaxN = (int64_t)1 << 31;  // exclusive

bool bad_dtype(int32_t dtype) { return dtype != APSP_I32 && dtype != APSP_F32; }

int32_t check_matrix(const void *dist, int64_t n, int64_t ld, int32_t dtype) {
    if (bad_dtype(dtype)) return APSP_ERR_INVALID_VALUE;
    if (n < 0 || n >= kMaxN) return APSP_ERR_INVALID_VALUE;
    if (ld < (n > 1 ? n : 1)) return APSP_ERR_INVALID_VALUE;
    if (n > 0 && dist == nullptr) return APSP_ERR_INVALID_VALUE;
    // n x ld elements of 4 bytes must be addressable: n * ld < 2^61
    if (n > 0 && ld > (((int64_t)1 << 61) / n)) return APSP_ERR_INVALID_VALUE;
    return APSP_OK;
}

// Working copy.  Two layouts make a solve slower than it needs to be:
//  * rows that are not 16-byte aligned (ld % 4 != 0, or a base address off
//    16 bytes) take the kernels' word-by-word load path: about 1.45x slower
//    (n = 8191: 24.3 against 16.7 ms; n = 16461: 177.5 against 124.2 ms);
//  * with rounds of 128 and n not a multiple of 128 the tiles of the last
//    block row and column are partial, and the operands cannot be staged
//    straight into LDS anywhere: 6-7 % slower than the same matrix padded to
//    a multiple of 128 with isolated vertices (n = 8300: 18.3 against
//    17.0 ms; n = 16461: 124.4 against 115.8 ms).  Below 64 rounds the
//    padding and the copies cost what the staging gains (n = 5200: 6.11
//    against 6.09 ms; n = 6000: 7.80 against 7.77 ms), so only matrices of 64
//    or more rounds are padded, and only by at most 1 % more vertices
//    (pads_to_128).
// From g_aligned_copy_min_n vertices such a call runs on a working copy: rows
// padded to 4 elements, and, for the second case, n padded to a multiple of
// 128 with vertices that have no edges (+inf, or 2^30, off the diagonal; 0 on
// it).  A vertex with no edges is no intermediate vertex of any path and its
// own entries stay "no edge" through every round, and the real vertices keep
// their blocks, so the rounds perform exactly the same operations on the real
// entries: the result is the same bits.  The copy is stream-ordered
// (hipMallocAsync on the caller's stream), filled and copied back by row-copy
// kernels (about 0.1 ms each way at n = 8192) and freed behind that work; a
// call of fewer than 16 rounds is not padded (the copies would cost more than
// the rounds gain), and without memory for the copy the call runs in place.
// Measured with the copy against in place, contiguous (unaligned) rows: n =
// 255 0.150 / 0.145 ms, 511 0.259 / 0.274, 2047 1.10 / 1.29, 8191 16.97 /
// 24.41, 16461 119.4 / 179.1; rows padded to 4 (padding to 128 only): 8300
// 17.70 / 18.45, 12000 47.40 / 50.11, 16461 119.2 / 126.9.
constexpr int64_t kDefaultAlignedCopyMinN = 512;
constexpr int64_t kPadMinRounds = 16;     // rounds in the call
constexpr int64_t kPadMinMatrixRounds = 64;  // rounds of the whole matrix
std::atomic<int64_t> g_aligned_copy_min_n{kDefaultAlignedCopyMinN};

// Whether a matrix of n vertices is worth padding to a multiple of 128: rounds
// of 128, 64 or more of them, and at most 1 % more vertices (up to about 3 %
// more work against the 6-7 % the staging gains: n = 8193, padded to 8320,
// measured 17.74 against 17.65 ms in place).
bool pads_to_128(int64_t n) {
    const int64_t b = apsp::round_width(n);
    if (b != apsp::kRoundB || n % b == 0 || (n + b - 1) / b < kPadMinMatrixRounds) return false;
    const int64_t extra = b - n % b;
    return 100 * extra <= n;
}

// The vertex count of the working copy of a call of `rounds` rounds on this
// matrix, or 0 when the call runs in place.
int64_t working_n(const void *dist, int64_t n, int64_t ld, int64_t rounds) {
    if (n <= 0 || n < g_aligned_copy_min_n.load()) return 0;
    const bool aligned = (reinterpret_cast<uintptr_t>(dist) & 15u) == 0 && (ld & 3) == 0;
    const bool pad = rounds >= kPadMinRounds && pads_to_128(n);
    if (aligned && !pad) return 0;
    const int64_t b = apsp::kRoundB;
    return pad ? (n + b - 1) / b * b : n;
}

// Run solve(ptr, n, ld) on the matrix itself or on its working copy (see
// above); the copy's result is copied back only when solve succeeds.
template <class F>
int32_t on_working_copy(void *dist, int64_t n, int64_t ld, int32_t dtype, int64_t rounds,
                        hipStream_t s, F &&solve) {
    const int64_t nw = working_n(dist, n, ld, rounds);
    if (nw == 0) return solve(static_cast<uint32_t *>(dist), n, ld);
    const int64_t ldw = (nw + 3) & ~(int64_t)3;
    uint32_t *w = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&w), (size_t)nw * (size_t)ldw * sizeof(uint32_t),
                       s) != hipSuccess) {
        (void)hipGetLastError();  // no room for the copy: solve in place
        return solve(static_cast<uint32_t *>(dist), n, ld);
    }
    uint32_t *d = static_cast<uint32_t *>(dist);
    const uint32_t none = dtype == APSP_I32 ? (uint32_t)APSP_INF_I32 : 0x7f800000u;
    hipError_t e = apsp::launch_copy_pad(w, ldw, nw, d, ld, n, none, s);
    int32_t st = APSP_ERR_DEVICE;
    if (e != hipSuccess) {
        apsp::note_error("working copy", e);
    } else {
        st = solve(w, nw, ldw);
        if (st == APSP_OK) {
            e = apsp::launch_copy_rows(d, ld, w, ldw, n, s);
            if (e != hipSuccess) {
                apsp::note_error("copy back from the working copy", e);
                st = APSP_ERR_DEVICE;
            }
        }
    }
    (void)hipFreeAsync(w, s);
    return st;
}

// Rounds r0 .. r1-1 clamped to the matrix's q.
int64_t call_rounds(int64_t n, int64_t r0, int64_t r1) {
    const int64_t b = apsp::round_width(n);
    const int64_t q = (n + b - 1) / b;
    const int64_t hi = r1 < q ? r1 : q;
    return hi > r0 ? hi - r0 : 0;
}

int32_t rounds_impl(void *dist, int64_t n, int64_t ld, int32_t dtype, int64_t r0, int64_t r1,
                    void *stream, apsp::PhaseTimes *times) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return on_working_copy(dist, n, ld, dtype, call_rounds(n, r0, r1), s,
                           [&](uint32_t *D, int64_t nD, int64_t ldD) -> int32_t {
        const hipError_t e = apsp::run_rounds(D, nD, ldD, dtype, r0, r1, r0 == 0, s, times);
        if (e == hipErrorOutOfMemory) return APSP_ERR_NO_MEMORY;
        return e == hipSuccess ? APSP_OK : APSP_ERR_DEVICE;
    });
}

}  // namespace

int64_t apsp::aligned_copy_min_n() { return g_aligned_copy_min_n.load(); }

extern "C" {

int32_t apsp_solve(void *dist, int64_t n, int64_t ld, int32_t dtype, void *stream) {
    const int32_t st = check_matrix(dist, n, ld, dtype);
    if (st != APSP_OK) return st;
    return rounds_impl(dist, n, ld, dtype, 0, INT64_MAX, stream, nullptr);
}

int32_t apsp_solve_rounds(void *dist, int64_t n, int64_t ld, int32_t dtype, int64_t r0,
                          int64_t r1, void *stream) {
    const int32_t st = check_matrix(dist, n, ld, dtype);
    if (st != APSP_OK) return st;
    if (r0 < 0 || r1 < 0) return APSP_ERR_INVALID_VALUE;
    return rounds_impl(dist, n, ld, dtype, r0, r1, stream, nullptr);
}

int32_t apsp_solve_profiled(void *dist, int64_t n, int64_t ld, int32_t dtype, void *stream,
                            double *phase_ms) {
    const int32_t st = check_matrix(dist, n, ld, dtype);
    if (st != APSP_OK) return st;
    if (phase_ms == nullptr) return APSP_ERR_INVALID_VALUE;
    apsp::PhaseTimes t;
    int32_t res = rounds_impl(dist, n, ld, dtype, 0, INT64_MAX, stream, &t);
    // synchronous, also when the result comes back from an aligned working copy
    if (res == APSP_OK && working_n(dist, n, ld, call_rounds(n, 0, INT64_MAX)) != 0) {
        const hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
        if (e != hipSuccess) {
            apsp::note_error("hipStreamSynchronize", e);
            res = APSP_ERR_DEVICE;
        }
    }
    for (int i = 0; i < 8; ++i) phase_ms[i] = (res == APSP_OK) ? t.ms[i] : 0.0;
    return res;
}

int32_t apsp_round_width(int64_t n, int32_t dtype) {
    return bad_dtype(dtype) ? 0 : apsp::round_width(n);
}

int64_t apsp_set_width64_max_n(int64_t n) {
    if (n < 0 || n > APSP_WIDTH64_MAX_N_LIMIT) return -1;
    return apsp::set_width64_max_n(n);
}

int64_t apsp_set_aligned_copy_min_n(int64_t n) {
    if (n < 0) return -1;
    return g_aligned_copy_min_n.exchange(n);
}

int64_t apsp_stream_state_bytes(int64_t n, int32_t dtype) {
    if (bad_dtype(dtype) || n < 0 || n >= kMaxN) return -1;
    // a full solve padded to a multiple of 128 keeps the state of the padded n
    const bool pad = n >= g_aligned_copy_min_n.load() && pads_to_128(n);
    const int64_t b = apsp::kRoundB;
    return apsp::stream_state_bytes(pad ? (n + b - 1) / b * b : n, dtype);
}

int64_t apsp_stream_state_count(void) { return apsp::stream_state_count(); }

int32_t apsp_release_stream_state(void *stream) {
    return apsp::release_stream_state(reinterpret_cast<hipStream_t>(stream)) == hipSuccess
               ? APSP_OK
               : APSP_ERR_DEVICE;
}

int32_t apsp_set_round_pair_threshold(int32_t rounds) {
    if (rounds < 2) return -1;
    return (int32_t)apsp::set_pair_rounds(rounds);
}

int32_t apsp_batched_round_width(int64_t n, int32_t dtype) {
    return bad_dtype(dtype) ? 0 : apsp::batched_tile(n);
}

int32_t apsp_minplus(void *C, int64_t ldc, const void *A, int64_t lda, const void *B, int64_t ldb,
                     int64_t m, int64_t n, int64_t k, int32_t dtype, int32_t accumulate,
                     void *stream) {
    if (bad_dtype(dtype) || m < 0 || n < 0 || k < 0) return APSP_ERR_INVALID_VALUE;
    if (m == 0 || n == 0) return APSP_OK;
    if (k == 0 || k >= kMaxN) return APSP_ERR_INVALID_VALUE;
    if (!C || !A || !B) return APSP_ERR_INVALID_VALUE;
    if (ldc < n || lda < k || ldb < n) return APSP_ERR_INVALID_VALUE;
    const int64_t tiles = ((m + apsp::kRoundB - 1) / apsp::kRoundB) *
                          ((n + apsp::kRoundB - 1) / apsp::kRoundB);
    if (tiles >= kMaxN) return APSP_ERR_INVALID_VALUE;
    // C must not overlap an operand: compare the address ranges spanned
    const uintptr_t c0 = reinterpret_cast<uintptr_t>(C);
    const uintptr_t c1 = c0 + 4 * (uintptr_t)((m - 1) * ldc + n);
    auto overlaps = [&](const void *p, int64_t rows, int64_t ld, int64_t cols) {
        const uintptr_t p0 = reinterpret_cast<uintptr_t>(p);
        const uintptr_t p1 = p0 + 4 * (uintptr_t)((rows - 1) * ld + cols);
        return p0 < c1 && c0 < p1;
    };
    if (overlaps(A, m, lda, k) || overlaps(B, k, ldb, n)) return APSP_ERR_INVALID_VALUE;
    const hipError_t e = apsp::launch_minplus(
        static_cast<uint32_t *>(C), ldc, static_cast<const uint32_t *>(A), lda,
        static_cast<const uint32_t *>(B), ldb, m, n, k, dtype, accumulate != 0,
        reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess) {
        apsp::note_error("min-plus product launch", e);
        return APSP_ERR_DEVICE;
    }
    return APSP_OK;
}

int32_t apsp_squarings(int64_t n) {
    int32_t s = 0;
    while (n > 2 && ((int64_t)1 << s) < n - 1) ++s;
    return s;
}

int32_t apsp_solve_squaring(void *dist, int64_t n, int64_t ld, int32_t dtype, void *work,
                            int64_t ldw, void *stream) {
    const int32_t st = check_matrix(dist, n, ld, dtype);
    if (st != APSP_OK) return st;
    if (n == 0) return APSP_OK;
    if (work == nullptr || ldw < n) return APSP_ERR_INVALID_VALUE;
    {
        const uintptr_t a0 = reinterpret_cast<uintptr_t>(dist);
        const uintptr_t a1 = a0 + 4 * (uintptr_t)((n - 1) * ld + n);
        const uintptr_t b0 = reinterpret_cast<uintptr_t>(work);
        const uintptr_t b1 = b0 + 4 * (uintptr_t)((n - 1) * ldw + n);
        if (a0 < b1 && b0 < a1) return APSP_ERR_INVALID_VALUE;
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint32_t *X = static_cast<uint32_t *>(dist), *Y = static_cast<uint32_t *>(work);
    int64_t ldx = ld, ldy = ldw;
    hipError_t e = apsp::launch_prologue(X, n, ld, dtype, s);
    const int32_t steps = apsp_squarings(n);
    for (int32_t i = 0; i < steps && e == hipSuccess; ++i) {
        // with a zero diagonal X (x) X <= X, so the product alone is the update
        e = apsp::launch_minplus(Y, ldy, X, ldx, X, ldx, n, n, n, dtype, false, s);
        std::swap(X, Y);
        std::swap(ldx, ldy);
    }
    if (e == hipSuccess && X != static_cast<uint32_t *>(dist))
        e = hipMemcpy2DAsync(dist, (size_t)ld * 4, X, (size_t)ldx * 4, (size_t)n * 4, (size_t)n,
                             hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
        apsp::note_error("repeated squaring", e);
        return APSP_ERR_DEVICE;
    }
    return APSP_OK;
}

int32_t apsp_solve_symmetric(void *dist, int64_t n, int64_t ld, int32_t dtype, void *stream) {
    const int32_t st = check_matrix(dist, n, ld, dtype);
    if (st != APSP_OK) return st;
    if (n == 0) return APSP_OK;
    if ((n + apsp::kRoundB - 1) / apsp::kRoundB > 46000) return APSP_ERR_INVALID_VALUE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return on_working_copy(dist, n, ld, dtype, (n + apsp::kRoundB - 1) / apsp::kRoundB, s,
                           [&](uint32_t *D, int64_t nD, int64_t ldD) -> int32_t {
        const hipError_t e = apsp::run_symmetric(D, nD, ldD, dtype, s);
        if (e == hipErrorOutOfMemory) return APSP_ERR_NO_MEMORY;
        return e == hipSuccess ? APSP_OK : APSP_ERR_DEVICE;
    });
}

int32_t apsp_validate(const void *dist, int64_t n, int64_t ld, int32_t dtype, void *stream) {
    const int32_t st = check_matrix(dist, n, ld, dtype);
    if (st != APSP_OK) return st;
    if (n == 0) return APSP_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    uint32_t *flag = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&flag), sizeof(uint32_t), s) != hipSuccess) {
        (void)hipGetLastError();
        return APSP_ERR_NO_MEMORY;
    }
    uint32_t host_flag = 0;
    int32_t result = APSP_OK;
    if (hipMemsetAsync(flag, 0, sizeof(uint32_t), s) != hipSuccess ||
        apsp::launch_validate(static_cast<const uint32_t *>(dist), n, ld, dtype, flag, s) !=
            hipSuccess ||
        hipMemcpyAsync(&host_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        result = APSP_ERR_DEVICE;
    else if (host_flag != 0)
        result = APSP_ERR_BAD_INPUT;
    (void)hipFreeAsync(flag, s);
    return result;
}

const char *apsp_status_string(int32_t status) {
    switch (status) {
    case APSP_OK: return "APSP_OK";
    case APSP_ERR_INVALID_VALUE: return "APSP_ERR_INVALID_VALUE: bad size, leading dimension, pointer, dtype or count";
    case APSP_ERR_UNSUPPORTED: return "APSP_ERR_UNSUPPORTED: request not supported by this library version";
    case APSP_ERR_DEVICE: return "APSP_ERR_DEVICE: a HIP call or kernel launch failed";
    case APSP_ERR_NO_MEMORY: return "APSP_ERR_NO_MEMORY: device workspace allocation failed";
    case APSP_ERR_BAD_INPUT: return "APSP_ERR_BAD_INPUT: negative weight or NaN in the matrix";
    default: return "APSP: unknown status";
    }
}

const char *apsp_version(void) { return "apsp-mi355x 0.1.0 gfx950"; }

const char *apsp_last_error(void) { return apsp::g_last_error; }

}  // extern "C"

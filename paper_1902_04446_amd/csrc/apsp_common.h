// Shared device helpers and internal launcher declarations of the APSP library.
//
// Element arithmetic of the min-plus (tropical) semiring used by every phase
// of the blocked method (arXiv:1902.04446, Table 1: MatProd is the (min, +)
// product, MatMin the element-wise minimum).  Both element types are carried
// as 32-bit words so one kernel body serves both:
//
//  * OpI32: int32 weights in [0, 2^30] computed as uint32.  Every stored value
//    stays <= 2^30 (a minimum always includes the current value), so a sum of
//    two is <= 2^31 and never wraps; v_add_u32 + v_min3_u32.
//  * OpF32: fp32 bit patterns.  Weights are >= 0 (or -0), and for such values
//    the signed-integer order of the bit patterns is the numeric order, with
//    +inf (0x7f800000) above every finite value.  Taking the minimum on the
//    bits (v_min3_i32) therefore equals the fp32 minimum and needs no NaN
//    canonicalisation; the sum is an IEEE fp32 add (v_add_f32).
//
// Neither form uses packed fp32 instructions.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <stdint.h>

struct apsp_batch_plan;  // opaque plan of the C ABI (apsp_batch_plan.hip)

namespace apsp {

constexpr uint32_t kInfI32 = 1u << 30;
constexpr uint32_t kInfF32Bits = 0x7f800000u;

struct OpI32 {
    static __device__ __forceinline__ uint32_t add(uint32_t a, uint32_t b) { return a + b; }
    static __device__ __forceinline__ uint32_t out(uint32_t v) { return v; }
    static __device__ __forceinline__ uint32_t min2(uint32_t a, uint32_t b) { return a < b ? a : b; }
    static __device__ __forceinline__ uint32_t min3(uint32_t a, uint32_t b, uint32_t c) {
        return min2(min2(a, b), c);
    }
    static __device__ __forceinline__ uint32_t pad() { return kInfI32; }
    // input normalisation: anything above 2^30 means "no edge"
    static __device__ __forceinline__ uint32_t norm(uint32_t v) { return v > kInfI32 ? kInfI32 : v; }
};

struct OpF32 {
    static __device__ __forceinline__ uint32_t add(uint32_t a, uint32_t b) {
        return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
    }
    static __device__ __forceinline__ uint32_t min2(uint32_t a, uint32_t b) {
        return (int32_t)a < (int32_t)b ? a : b;
    }
    static __device__ __forceinline__ uint32_t min3(uint32_t a, uint32_t b, uint32_t c) {
        return min2(min2(a, b), c);
    }
    static __device__ __forceinline__ uint32_t pad() { return kInfF32Bits; }
    static __device__ __forceinline__ uint32_t norm(uint32_t v) { return v; }
    static __device__ __forceinline__ uint32_t out(uint32_t v) { return v; }
};

//  * OpI32F: int32 storage, fp32 arithmetic.  Values are converted as they
//    are loaded ((float)min(v, 2^30): "no edge" stays the finite 2^30) and
//    back as they are stored (min(v, 2^30) of the integer value).  A sum with
//    a "no edge" term is at least 2^30, above every path length (< 2^24), so
//    it never wins a minimum against one and is stored as 2^30; stored
//    values only decrease, so no sum exceeds 2^31 (exact in fp32).  Padding
//    outside the matrix is +inf.  Exact whenever every sum of two path lengths
//    the method forms is an integer below 2^24.  Every value the blocked method stores is the length
//    of a shortest path over some subset of intermediate vertices, so at most
//    (n-1) * wmax for the largest finite weight wmax, and every sum it forms
//    adds two of them: 2 (n-1) wmax < 2^24 is sufficient (int_exact_in_f32).
//    The same holds when a solve resumes from a partial state, with wmax the
//    largest finite entry of that state: the remaining rounds compute shortest
//    paths over subsets of intermediate vertices of the graph it describes.
//    fp32 adds issue at a higher rate than uint32 adds on this VALU.
struct OpI32F {
    static __device__ __forceinline__ uint32_t add(uint32_t a, uint32_t b) {
        return __float_as_uint(__uint_as_float(a) + __uint_as_float(b));
    }
    static __device__ __forceinline__ uint32_t min2(uint32_t a, uint32_t b) {
        return (int32_t)a < (int32_t)b ? a : b;
    }
    static __device__ __forceinline__ uint32_t min3(uint32_t a, uint32_t b, uint32_t c) {
        return min2(min2(a, b), c);
    }
    static __device__ __forceinline__ uint32_t pad() { return kInfF32Bits; }
    static __device__ __forceinline__ uint32_t norm(uint32_t v) {
        return __float_as_uint((float)(v < kInfI32 ? v : kInfI32));
    }
    static __device__ __forceinline__ uint32_t out(uint32_t v) {
        const uint32_t x = (uint32_t)__uint_as_float(v);
        return x < kInfI32 ? x : kInfI32;
    }
};

// Whether a graph of n vertices whose largest finite off-diagonal entry is
// wmax may take the OpI32F path bit-exactly: 2 (n-1) wmax < 2^24.
__host__ __device__ __forceinline__ bool int_exact_in_f32(int64_t n, uint32_t wmax) {
    return n <= 1 || (uint64_t)2 * (uint64_t)(n - 1) * wmax < (1u << 24);
}

// Round width of the single-graph solver and the output tile of the
// phase-2/phase-3 kernels (one workgroup per 128 x 128 tile).
constexpr int kRoundB = 128;

// Per-graph descriptor of a batched solve (tile: the graph's round width, 64
// or 128).
struct BatchDesc {
    uint32_t *ptr;
    int64_t ld;
    int32_t n;
    int32_t tile;
};

// One workgroup's work in a batched launch: tile (I, J) = (ij >> 16, ij & 0xffff)
// of graph `graph`.
struct BatchItem {
    int32_t graph;
    int32_t ij;
};

// Items of a batched launch, grouped by the XCD their workgroups run on
// (workgroup w runs on XCD w % 8): XCD x takes items offset[x] .. +count[x].
struct XcdRanges {
    int32_t offset[8];
    int32_t count[8];
};

// Tile sets of the min-plus tile kernel (round r, q rounds):
constexpr int kPanels = 0;  // phase 2: block row r and block column r, 2(q-1) tiles
constexpr int kAll = 1;     // phase 3: every tile outside block row/column r, (q-1)^2
constexpr int kNext = 2;    // phase 3, tiles in block row/column r+1, 2q-3
constexpr int kRest = 3;    // phase 3, tiles outside block rows/columns r, r+1, (q-2)^2

// ---- launchers (host side; each returns a hipError_t) ----------------------
hipError_t launch_prologue(uint32_t *D, int64_t n, int64_t ld, int dtype, hipStream_t s);
// dst[i * ldd + j] = src[i * lds + j] for i, j < n (the matrices must not overlap).
// launch_copy_pad: the same for an nd x nd dst (nd >= n), whose vertices n ..
// nd-1 get no edges (`none` off the diagonal, 0 on it).
hipError_t launch_copy_rows(uint32_t *dst, int64_t ldd, const uint32_t *src, int64_t lds, int64_t n,
                            hipStream_t s);
hipError_t launch_copy_pad(uint32_t *dst, int64_t ldd, int64_t nd, const uint32_t *src,
                           int64_t lds, int64_t n, uint32_t none, hipStream_t s);
// A batched graph's working copy: `user` (leading dimension ld_user) and
// `work` (ld_work, 16-byte rows); its rows are rows row0 .. row0+n-1 of the
// copy launch.
struct BatchCopy {
    uint32_t *user;
    uint32_t *work;
    int64_t ld_user, ld_work;
    int64_t row0;
    int32_t n, pad_;
};
// Copy every listed graph into its working copy (back == false) or back
// (back == true); `rows` is the sum of their n.  Entries in row0 order.
hipError_t launch_batch_copies(const BatchCopy *copies, int32_t count, int64_t rows, bool back,
                               hipStream_t s);
// Threshold of the working copies (apsp_set_aligned_copy_min_n).
int64_t aligned_copy_min_n();
// dtype of the kernels that run an int32 matrix held as the fp32 bits of
// OpI32F (when its wmax word allows the fp32 pipe; as uint32 otherwise):
// those kernels compute as OpF32 (or OpI32) and convert nothing.
// launch_conv_i32 converts such a matrix in place, in (to_f32) or back.
constexpr int kI32AsF32 = 2;
hipError_t launch_conv_i32(uint32_t *D, int64_t n, int64_t ld, const uint32_t *wmax, bool to_f32,
                           hipStream_t s);
// wmax: the int32 word (dtype kI32AsF32 only)
hipError_t launch_phase1(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, hipStream_t s,
                         const uint32_t *wmax = nullptr);
// close_next_diag (kNext only): the workgroup of diagonal block r+1 also runs
// phase 1 of round r+1 on it before storing it.
// wmax (int32 only): the word launch_wmax filled for this matrix; int32 tiles
// then run on the fp32 pipe when int_exact_in_f32(n, *wmax), else in uint32.
hipError_t launch_tile_set(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, int set,
                           hipStream_t s, bool close_next_diag = false,
                           const uint32_t *wmax = nullptr);
// *wmax = largest finite (< 2^30) off-diagonal entry of the int32 matrix.
hipError_t launch_wmax(const uint32_t *D, int64_t n, int64_t ld, uint32_t *wmax, hipStream_t s);
// Phase-3 tiles outside block rows/columns r, r+1 whose block row lies in
// [lo, hi) (kRest restricted to a band of block rows), and their count.
hipError_t launch_rest_rows(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, int64_t lo,
                            int64_t hi, hipStream_t s, const uint32_t *wmax = nullptr);
int64_t rest_rows_count(int64_t n, int64_t r, int64_t lo, int64_t hi);
int64_t num_rounds(int64_t n);

// ---- width-64 rounds for small matrices (apsp_small.hip) --------------------
// The single-graph solver's round width for an n-vertex matrix: 64 up to a
// process-wide limit (set_width64_max_n), else kRoundB.
int round_width(int64_t n);
int64_t set_width64_max_n(int64_t n);
int64_t num_rounds64(int64_t n);
// Phase 1 of round r at width 64.
hipError_t launch_phase1_64(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                            hipStream_t s);
// A phase-2/3 tile set of round r at width 64 (kRest: block rows [lo, hi)).
hipError_t launch_tile_set64(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, int set,
                             hipStream_t s, bool close_next_diag, const uint32_t *wmax,
                             int64_t lo, int64_t hi);

// ---- round pairs (apsp_pair.hip) -------------------------------------------
// Copies of round panels, all with leading dimension ld = 128 q (q rounds):
// row[s] holds a block row (its row k at offset k * ld); colT[s] a block
// column stored transposed (the block's column k at offset k * ld, matrix row
// i at position i), the layout the direct-staged rest pass takes its A operand
// in.  Phase 2 of a pair's second round writes row[s] and colT[s] for s in a
// three-slot ring (a pass may still read the previous pair's copies while the
// next pair writes its own); phase 2 of a pair's first round writes colT[3]
// or colT[4], alternating between pairs.
constexpr int kPairRowSlots = 3;
constexpr int kPairFirstSlot0 = 3;  // colT slots 3, 4: the pair's first round
struct PairCopies {
    uint32_t *row[kPairRowSlots] = {};
    uint32_t *colT[5] = {};
    int64_t ld = 0;
};
// Blocks r+2, r+3 that exist (0..2): the next pair's.
int pair_next_blocks(int64_t n, int64_t r);
// Phase 2 of round pr, also written to the copies: block row to row[row_slot]
// (none when row_slot < 0), block column transposed to colT[col_slot].
hipError_t launch_pair_panels(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t pr,
                              const PairCopies &c, int row_slot, int col_slot, hipStream_t s,
                              const uint32_t *wmax);
// Round r's phase 3 on block row/column r+1 (the tiles round r+1 reads
// first), closing diagonal block r+1 after its update: launch_tile_set(kNext)
// with the fused closure, or its direct-staged form (as launch_pair_rest),
// the column panel of round r read from colT[first_slot].
hipError_t launch_pair_round_next(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                                  const PairCopies &c, int first_slot, hipStream_t s,
                                  const uint32_t *wmax);
// Phase 3 of rounds r and r+1 on the tiles of block rows/columns r+2, r+3
// outside blocks r, r+1; `close` closes diagonal block r+2 after its update.
// prev >= 0: tiles of block row/column prev (but prev+1) first take round
// prev+1's deferred update from copy slot prev_slot (row and colT).  The
// column panels of rounds r and r+1 are in colT[first_slot] and colT[slot]
// (read by the direct-staged kernel; see launch_pair_rest).
hipError_t launch_pair_next(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                            bool close, int64_t prev, const PairCopies &c, int prev_slot,
                            int first_slot, int slot, hipStream_t s, const uint32_t *wmax);
// Phase 3 of rounds r and r+1 on the tiles outside blocks r .. r+1+next
// whose block row is in [lo, hi); deferred updates as launch_pair_next.  The
// column panels of rounds r and r+1 are in colT[first_slot] and colT[slot]
// (read by the direct-staged kernels, which full tiles of aligned fp32
// matrices, and of aligned int32 matrices held as kI32AsF32, take; the other
// kernels read them from the matrix).
hipError_t launch_pair_rest(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                            int64_t lo, int64_t hi, int64_t prev, const PairCopies &c,
                            int prev_slot, int first_slot, int slot, hipStream_t s,
                            const uint32_t *wmax);
int64_t pair_rest_count(int64_t n, int64_t r, int64_t lo, int64_t hi);
// Whether launch_pair_rest takes the direct-staged kernel for this matrix.
bool pair_rest_direct(const uint32_t *D, int64_t n, int64_t ld, int dtype);
// A single round's rest set on block rows [lo, hi) (outside block rows/columns
// r, r+1), direct-staged: fp32 or kI32AsF32 (wmax its word), with
// pair_rest_direct(D, ...) true, the column panel of round r transposed in
// c.colT[col_slot] (launch_pair_panels).
hipError_t launch_round_rest_direct(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r,
                                   int64_t lo, int64_t hi, const PairCopies &c, int col_slot,
                                   hipStream_t s, const uint32_t *wmax);
// Round r+1's deferred phase-3 update on block row/column r: !final_: tiles
// (x, r), (r, x) for the next blocks x; final_: every other one but the
// blocks r+1.
hipError_t launch_pair_fix(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r, bool final_,
                           hipStream_t s, const uint32_t *wmax);
int64_t tile_count(int64_t n, int64_t r, int set);
hipError_t launch_validate(const uint32_t *D, int64_t n, int64_t ld, int dtype, uint32_t *flag,
                           hipStream_t s);
// Batched launches (apsp_batched.hip).  `wmax` (int32
// batches) holds each graph's largest finite weight, from launch_batched_wmax,
// which zeroes it and scans the 128 x 128 tiles given by its items.
hipError_t launch_batched_wmax(const BatchDesc *descs, const BatchItem *items,
                               const XcdRanges &ranges, uint32_t *wmax, int32_t graphs,
                               hipStream_t s);
hipError_t launch_batched_items(const BatchDesc *descs, const BatchItem *items,
                                const XcdRanges &ranges, int r, bool close_only, int dtype,
                                const uint32_t *wmax, hipStream_t s);
// Batched round width (64 or 128) for a graph of n vertices, from the
// batched tuning table (apsp_autotune.hip).
int batched_tile(int64_t n);
constexpr int kTuneBuckets = 9;  // bucket b < 8: n in (64b, 64b + 64]; bucket 8: n > 512
int batched_bucket(int64_t n);
// The current device's batched width of every bucket (kTuneBuckets entries;
// 128 everywhere without a device).
void batched_tuning_snapshot(int32_t *table);
// Plan with the round width of each graph taken from `table` (kTuneBuckets
// entries, 64 or 128), for the batched autotuner; arguments as
// apsp_batched_plan_create.
int32_t batched_plan_create_table(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                  int32_t count, int32_t dtype, const int32_t *table,
                                  hipStream_t s, ::apsp_batch_plan **out);

// C = A (x) B, or C = min(C, A (x) B) when accumulate; C is m x n, A m x k,
// B k x n, row-major with the given leading dimensions; C must not overlap
// A or B.  k == 0 gives "no edge" everywhere (or leaves C as it is).
hipError_t launch_minplus(uint32_t *C, int64_t ldc, const uint32_t *A, int64_t lda,
                          const uint32_t *B, int64_t ldb, int64_t m, int64_t n, int64_t k,
                          int dtype, bool accumulate, hipStream_t s);

// Symmetric variant (upper-triangle blocks only, lower filled at the end).
hipError_t run_symmetric(uint32_t *D, int64_t n, int64_t ld, int dtype, hipStream_t s);

// Record the failing HIP call of the current thread (apsp_last_error()).
void note_error(const char *what, hipError_t e);
// Record a message for apsp_last_error() (a request the library refused).
void note_message(const char *what);

// ---- round scheduler (apsp_runtime.hip) ------------------------------------
// Per-phase elapsed milliseconds of a profiled solve (see apsp_solve_profiled).
struct PhaseTimes {
    double ms[8];
};
// Enqueue rounds r0..r1-1 (r1 clamped to q) on stream s, with the input
// normalisation first when `prologue`.  `times` (nullable) requests event
// timing; the call then waits for completion before filling it in.
hipError_t run_rounds(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r0, int64_t r1,
                      bool prologue, hipStream_t s, PhaseTimes *times);
// Rounds from which run_rounds uses round pairs; returns the previous value.
int64_t set_pair_rounds(int64_t rounds);
// Per-(device, caller stream) state of run_rounds: its device bytes after a
// full solve of n on a fresh stream, how many states exist, and releasing the
// state of `s` on the current device (waits for its work first).
int64_t stream_state_bytes(int64_t n, int dtype);
int64_t stream_state_count();
hipError_t release_stream_state(hipStream_t s);
// Part of that state lent to the symmetric solver: the chain stream and the
// first helper stream of caller stream s on the current device, four events
// and the first two row-copy slots (128 x ld words each, ld = 128 ceil(n /
// 128)), created on first use.  On hipSuccess *lock holds the state's
// enqueue lock.
struct SideResources {
    hipStream_t chain, side;
    hipEvent_t enter, leave, p2_done, rest_done;
    uint32_t *slot[2];
    int64_t ld;
};
hipError_t side_resources(hipStream_t s, int64_t n, SideResources *out,
                          std::unique_lock<std::mutex> *lock);

}  // namespace apsp

/*
 * apsp.h -- all-pairs shortest-path lengths on one AMD Instinct MI355X (gfx950).
 *
 * Method: blocked Floyd-Warshall in three phases per round (Schoeneman & Zola,
 * arXiv:1902.04446, Sec. 4.4 "Blocked In-Memory" and Sec. 4.5 "Blocked
 * Collect/Broadcast", Algorithms 3 and 4; the phase operations are Table 1's
 * FloydWarshall, MinPlus = MatProd followed by MatMin).  The problem is the
 * one stated in Sec. 3: an undirected weighted graph with no negative cycles,
 * vertices numbered 0..n-1, adjacency matrix A with A_ij = A_ji = w_ij, and
 * the output is the length of a shortest path between every pair (no paths).
 * Dropping the symmetry assumption gives the directed case (Sec. 4), which
 * this library also accepts: it never relies on A being symmetric.
 *
 * Matrix format (every entry point):
 *   - dense, row-major, n x n, leading dimension ld >= n (in elements),
 *     resident in device memory of the current HIP device;
 *   - element type APSP_I32 (int32) or APSP_F32 (fp32);
 *   - entry (i, j) is the weight of edge i->j; a missing edge is
 *       APSP_I32: any value >= APSP_INF_I32 (2^30),
 *       APSP_F32: +inf;
 *   - weights must be >= 0 (in an undirected graph a negative edge is a
 *     negative cycle); NaN is not allowed.  apsp_validate() checks this.
 *     Results for inputs outside this domain are unspecified (no fault).
 *   - the input diagonal is ignored: the empty path gives D_ii = 0.
 * Result, in place: D_ij = shortest-path length from i to j; unreachable
 * pairs hold APSP_INF_I32 (int32) or +inf (fp32).  int32 lengths that would
 * reach 2^30 or more are reported as APSP_INF_I32.  int32 results are exact;
 * fp32 results use IEEE round-to-nearest additions, one per path edge.
 *
 * Stream semantics: every call enqueues its work on `stream` (a hipStream_t;
 * NULL = the default stream) and returns before the work completes, except
 * apsp_validate(), which waits for its own result.  Host arrays passed in may
 * be reused as soon as a call returns.  The caller owns all device memory it
 * passes in; the library keeps no pointer to it after the enqueued work ends.
 *
 * Errors: arguments are checked on the host before any HIP call; a failed
 * check returns a status and enqueues nothing.  No C++ exception crosses this
 * interface.  Faults of the device work itself surface at the caller's next
 * synchronisation with `stream`.
 */
#ifndef APSP_H_
#define APSP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types (pass as the int32_t `dtype` argument). */
enum { APSP_I32 = 0, APSP_F32 = 1 };

/* Status codes. */
enum {
    APSP_OK = 0,
    APSP_ERR_INVALID_VALUE = 1, /* bad size, leading dimension, pointer, dtype or count */
    APSP_ERR_UNSUPPORTED = 2,   /* valid request this library version cannot serve */
    APSP_ERR_DEVICE = 3,        /* a HIP call or kernel launch failed */
    APSP_ERR_NO_MEMORY = 4,     /* device workspace could not be allocated */
    APSP_ERR_BAD_INPUT = 5      /* apsp_validate(): negative weight or NaN found */
};

/* Sentinel for "no edge" / "unreachable" in int32 matrices. */
#define APSP_INF_I32 (1 << 30)

/*
 * apsp_solve -- solve one graph in place (Sec. 4.4/4.5, all q = ceil(n/b)
 * rounds of the blocked method; b = apsp_round_width()).
 *   dist   device pointer to the n x n matrix (ld elements per row); may be
 *          NULL only when n == 0.
 *   n      number of vertices, 0 <= n <= 2^31 - 1 (n == 0: no-op).
 *   ld     leading dimension in elements, ld >= max(n, 1).
 *   dtype  APSP_I32 or APSP_F32.
 *   stream hipStream_t to enqueue on (NULL = default stream).
 * Rounds are 64 wide up to n = 5120 and 128 wide above (apsp_round_width).
 * From 3 rounds of 128 on (64 rounds of 64) the phases of round r+1 overlap
 * the bulk of round r's phase 3 on library-owned streams (one set per device
 * and caller stream, created on first use and kept until
 * apsp_release_stream_state): a chain stream, which waits for `stream`'s
 * earlier work and runs the chain of phases, and two band streams, created
 * one after the other so that HIP deals the three to different hardware
 * queues; from 64 rounds up that phase 3 runs as two bands of block rows on
 * the band streams.  The call makes `stream` wait for all of that work, so
 * stream order is preserved.  int32 matrices are first scanned for
 * their largest finite entry w; when 2 (n-1) w < 2^24 every sum the method
 * forms is an integer below 2^24, and the tiles are computed in fp32
 * arithmetic (exact, so the result is the same) at its higher issue rate.
 * The scan's result lives in a 256-byte device word allocated with the
 * helper streams.  From 64 rounds of 128, for calls of 16 or more rounds
 * on 16-byte aligned rows with n a multiple of 128 (or their working copy),
 * the call holds the int32 matrix as those fp32 values (converted in place
 * after the scan, back at the end of the call) and runs the fp32 kernels,
 * operands staged straight into LDS, or, when the scan rules the fp32 pipe
 * out, the same kernels in uint32 on the untouched words.  The matrix holds
 * int32 values again when the call's work is done.  From 72 rounds up (n > 9088; apsp_set_round_pair_threshold),
 * phase 3 runs in pairs of rounds: one pass per tile with k over both rounds' blocks, the second
 * round's update of the first round's block row and column deferred and
 * applied from a copy of its panels (the result is the same, bit for bit).
 * For fp32 matrices with n a multiple of 128 and 16-byte aligned rows,
 * phase 2 of every round of 128 also writes its block column transposed, and
 * the bulk of phase 3 reads it, in pairs or in single rounds (the operands
 * then go straight from memory into LDS).  The copies take 8 x 128 x 128q x 4
 * bytes (32 MiB at n = 8192, 64 MiB at n = 16384, 1 GiB at n = 262144),
 * allocated with the helper streams on first need and grown for a larger n;
 * growing synchronises `stream` and the helper streams inside the call
 * (solves still running on them may read the old copies).  When they cannot
 * be allocated the call runs single rounds without them.
 * Working copy.  Rows that are not 16-byte aligned (ld not a multiple of 4,
 * or dist not on 16 bytes) would take the kernels' word-by-word load path,
 * about 1.45x slower; rounds of 128 with n not a multiple of 128 run 6-7 %
 * slower than the same matrix padded to a multiple of 128.  From n = 512
 * (apsp_set_aligned_copy_min_n) such a call runs on a working copy: rows
 * padded to 4 elements and, for a matrix of 64 or more rounds of 128
 * (n > 8064) and a call of 16 or more rounds, n padded to a multiple of 128
 * with vertices that have no edges (which changes no operation on the real
 * entries) when that adds at most 1 % to n.  The copy (at most n' x n' words, n' the
 * padded n) comes from hipMallocAsync on `stream`, is filled, solved and
 * copied back in stream order, and is freed with hipFreeAsync behind that
 * work; when it cannot be allocated the call runs in place.  The result is
 * the same, bit for bit, either way.
 * Nothing else is allocated.
 * Solves enqueued on the same stream from several host threads are
 * serialised by the library.
 * Returns APSP_OK, APSP_ERR_INVALID_VALUE, APSP_ERR_NO_MEMORY (helper stream
 * could not be created) or APSP_ERR_DEVICE.
 */
int32_t apsp_solve(void *dist, int64_t n, int64_t ld, int32_t dtype, void *stream);

/*
 * apsp_set_round_pair_threshold -- the number of rounds q = ceil(n/b) from
 * which apsp_solve, apsp_solve_rounds (for a call of two or more rounds) and
 * apsp_solve_profiled run phase 3 in pairs of rounds (see apsp_solve;
 * default 72: measured on MI355X, pairs lose 6% at 64 rounds, where the
 * pair's longer chain of launches on the caller's stream is not hidden, and
 * win 2% at 72 and 7% at 128).  The results are the same either way.
 * rounds >= 2; pairs need at least 3 rounds whatever the threshold (with
 * 2 there is no rest set to pair); a value above any q disables pairs.
 * Process-wide, takes effect for solves enqueued afterwards; no HIP call.
 * Returns the previous threshold, or -1 (unchanged) when rounds < 2.
 */
int32_t apsp_set_round_pair_threshold(int32_t rounds);

/*
 * Per-stream state.  apsp_solve, apsp_solve_rounds, apsp_solve_profiled and
 * apsp_solve_symmetric keep, per (device, caller stream), the state
 * apsp_solve describes: three helper streams, five events, the 256-byte scan
 * word and, once a solve ran round pairs or a symmetric solve of 2 or more
 * rounds ran, the panel copies.  int32 solves and solves long enough for the
 * lookahead create it; it lives until released here or the process ends.
 *
 * apsp_stream_state_bytes -- device bytes of that state after a full
 * apsp_solve of an n-vertex `dtype` matrix on a stream without state: 0 when
 * such a solve creates none, else 256 plus the copies when it runs round
 * pairs (at the current thresholds).  (apsp_solve_symmetric of n > 128 keeps
 * 256 plus the copies for n.)  A stream's copies grow to its largest solve
 * and never shrink.  No HIP call.  Returns -1 for a bad dtype or n out of
 * range.
 *
 * apsp_stream_state_count -- how many (device, stream) states the process
 * holds.  No HIP call.
 *
 * apsp_release_stream_state -- release the state of `stream` (NULL = the
 * default stream) on the current device: blocks until all work enqueued on
 * `stream` and on its helper streams has finished, then destroys the helper
 * streams and events and frees the word and the copies.  A later solve on the
 * stream creates them again.  Call it before destroying a stream the library
 * solved on (a new stream may get the old handle) and when a stream is done
 * with large solves; it must not run concurrently with a solve enqueued on
 * the same stream from another thread.  Returns APSP_OK (also when the stream
 * has no state) or APSP_ERR_DEVICE (a synchronisation failed; the state is
 * kept).
 */
int64_t apsp_stream_state_bytes(int64_t n, int32_t dtype);
int64_t apsp_stream_state_count(void);
int32_t apsp_release_stream_state(void *stream);

/*
 * apsp_solve_rounds -- run rounds r0 .. r1-1 of the blocked method only
 * (Sec. 4.4: each round is phase 1 on diagonal block r, phase 2 on its block
 * row and block column, phase 3 on every other block).  r0 == 0 also applies
 * the input normalisation (zero diagonal, int32 entries above 2^30 mapped to
 * 2^30).  After rounds 0..r-1 the matrix equals Floyd-Warshall stopped after
 * pivots 0 .. min(r*b, n)-1, so a solve may be split into slices, checkpointed
 * and resumed between calls.  r1 is clamped to q; r0 >= r1 is a no-op.
 * Returns as apsp_solve; r0 < 0 or r1 < 0 is APSP_ERR_INVALID_VALUE.
 */
int32_t apsp_solve_rounds(void *dist, int64_t n, int64_t ld, int32_t dtype, int64_t r0,
                          int64_t r1, void *stream);

/*
 * apsp_solve_profiled -- apsp_solve with HIP events recorded around every
 * launch; waits for the solve to finish, then writes into phase_ms[0..7]:
 *   [0] input normalisation (ms)
 *   [1] phase 1, summed over rounds        [2] phase 2, summed over rounds
 *   [3] phase 3: [5] + [7]                 [4] the whole solve
 *   [5] the time during which the bulk of phase 3 was being updated (the
 *       tiles outside block rows/columns r .. r+3 of a pair of rounds, or
 *       outside r, r+1 of a single round): it runs as bands of block rows on
 *       helper streams, bands of consecutive pairs or rounds overlapping,
 *       and [5] is the union of those launches' intervals
 *   [6] how many pairs of rounds (or single rounds) had such launches
 *   [7] the other phase-3 launches on `stream` (block rows/columns r+1 ..
 *       r+3 and the deferred updates), summed
 * Phase-3 launches overlap phases 1 and 2 of the next round (one-round
 * lookahead), so [1] + [2] + [3] can exceed [4].  When the call runs on a
 * working copy (see apsp_solve) the phases time the solve on the copy, and
 * the copies in and back are outside them.  The result in `dist` is
 * identical to apsp_solve's.  phase_ms must have room for 8 values.
 * Synchronous.  Returns as apsp_solve.
 */
int32_t apsp_solve_profiled(void *dist, int64_t n, int64_t ld, int32_t dtype, void *stream,
                            double *phase_ms);

/*
 * apsp_solve_symmetric -- apsp_solve for an undirected graph (Sec. 3:
 * A_ij = A_ji) using only the upper-triangular blocks, as the paper stores
 * them (Sec. 4): phases 2 and 3 update blocks (I, J) with I <= J, reading the
 * transposes of upper blocks where the method needs a lower one; the strict
 * lower triangle is then filled from the upper one.  Only the upper triangle
 * of the input is read (the lower is overwritten).  Rounds are 128 wide.
 * For a symmetric input the result equals the 128-wide blocked method's bit
 * for bit (fp32 addition commutes; apsp_solve's whenever apsp_round_width(n)
 * is 128), with about half of its phase-2/3 work.  Phase 2 also writes block
 * row r whole into a copy (the row blocks as they are, the column blocks
 * transposed: by symmetry both are row r), from which phase 3 reads both of
 * its operands.  From 3 rounds on, the bulk of each round's phase 3 runs on
 * a helper stream of `stream` while phases 1 and 2 of the next round run on
 * `stream`, as in apsp_solve.  From 2 rounds on the call uses the per-stream
 * state of apsp_solve (helper streams, and the panel copies, of which it
 * uses two slots: 256 + 8 x 128 x 128q x 4 bytes, allocated or grown as
 * described there).  Layouts that would be slow get the working copy of
 * apsp_solve (from n = 512; the whole matrix copied in and back).
 * Asynchronous.  Returns as apsp_solve, or
 * APSP_ERR_NO_MEMORY when the copies cannot be allocated.
 */
int32_t apsp_solve_symmetric(void *dist, int64_t n, int64_t ld, int32_t dtype, void *stream);

/* Round width b used by apsp_solve / apsp_solve_rounds / apsp_solve_profiled
 * for an n-vertex matrix: 64 for n <= the width-64 limit (default 5120;
 * apsp_set_width64_max_n), 128 above it; q = ceil(n / b) rounds.  Sec. 4
 * leaves b to the user or a tuner.  Small solves are bound by the chain of
 * dependent launches of each round, which 64-wide rounds shorten.  int32
 * results do not depend on b; fp32 results are the blocked method's with
 * this b (every candidate is one IEEE addition, but phase 1 closes a b x b
 * block in pivot order, so the last bits may differ between widths).
 * Returns 0 for a bad dtype. */
int32_t apsp_round_width(int64_t n, int32_t dtype);

/* apsp_set_width64_max_n -- the largest n that apsp_solve and its variants
 * solve in rounds of width 64 (0 disables them; at most
 * APSP_WIDTH64_MAX_N_LIMIT).  Process-wide, for solves enqueued afterwards;
 * no HIP call.  A solve split over apsp_solve_rounds calls must not change
 * it between its calls.  Returns the previous value, or -1 (unchanged) for
 * n < 0 or n > APSP_WIDTH64_MAX_N_LIMIT. */
#define APSP_WIDTH64_MAX_N_LIMIT 8192
int64_t apsp_set_width64_max_n(int64_t n);

/* apsp_set_aligned_copy_min_n -- the smallest n from which apsp_solve,
 * apsp_solve_rounds (each call), apsp_solve_profiled and apsp_solve_symmetric
 * run on a working copy (see apsp_solve: rows not 16-byte aligned, or n not
 * a multiple of 128 with rounds of 128; default 512; a value above every n
 * turns the copy off).  A value above APSP_BATCHED_MAX_N also turns off the
 * batched working copies (see the batched plans).  Process-wide, for calls
 * made afterwards (and plans created afterwards); no HIP call.  Returns the
 * previous value, or -1 (unchanged) when n < 0. */
int64_t apsp_set_aligned_copy_min_n(int64_t n);

/*
 * apsp_solve_batched -- solve `count` independent int32 graphs together.
 *   ptrs[g]  device pointer to graph g's n_g x n_g int32 matrix (ld = n_g),
 *            solved in place; graphs must not overlap in memory.
 *   ns[g]    n_g, 0 <= n_g <= APSP_BATCHED_MAX_N.
 *   count    number of graphs, >= 0 (0: no-op; ptrs/ns may then be NULL).
 * Every graph goes through the rounds of the blocked method (Sec. 4.4/4.5)
 * with its own round width b_g = apsp_batched_round_width(n_g) (64 or 128);
 * each launch covers one phase of round r for every graph that has a round
 * r at its width (1 + 2 * max_g ceil(n_g / b_g) launches).  int32 results
 * are exactly apsp_solve's.  Builds a one-shot plan: its tables are
 * copied to stream-ordered device memory (hipMallocAsync) and freed
 * stream-ordered after the launches.
 * Returns APSP_OK, APSP_ERR_INVALID_VALUE, APSP_ERR_NO_MEMORY or
 * APSP_ERR_DEVICE.
 */
#define APSP_BATCHED_MAX_N 4096
int32_t apsp_solve_batched(void *const *ptrs, const int32_t *ns, int32_t count, void *stream);

/*
 * apsp_solve_batched_ex -- as apsp_solve_batched with per-graph leading
 * dimensions (lds[g] >= max(n_g, 1); lds == NULL means ld = n) and a dtype
 * for the whole batch.  fp32 graphs use the batched round width, so their
 * last bits may differ from apsp_solve's when that width differs; both are
 * the blocked method in IEEE fp32.
 */
int32_t apsp_solve_batched_ex(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                              int32_t count, int32_t dtype, void *stream);

/*
 * apsp_solve_batched_noalloc -- apsp_solve_batched_ex for callers that cannot
 * allocate device memory (code enqueued in tight serving loops, harnesses
 * that forbid hipMalloc): same arguments, same kernels, same results, but
 * the descriptor and work-item tables go to a fixed device workspace of
 * APSP_NOALLOC_WORKSPACE_BYTES that the library holds on every GPU it runs
 * on (a file-scope device array, kept until the process ends) instead of
 * stream-ordered allocations.  No hipMalloc, hipFree or other device
 * allocation is made.  The host tables are built in per-thread host buffers
 * that keep their size between calls.
 * Limit: the tables take 24 bytes per non-empty graph, 4 more per graph for
 * int32, rounded up to 16, plus 8 bytes per work item, where a graph with
 * q = ceil(n / b) rounds at its batched width b has 1 + q (q^2 - 1) items
 * (int32 adds ceil(n / 128)^2 for the weight scan).  A batch whose tables do
 * not fit is refused with APSP_ERR_UNSUPPORTED before any HIP call (the
 * 4096-graph batch of n <= 512 needs about 0.7 MiB); apsp_last_error() then
 * states the size needed.
 * Every call on a GPU uses that GPU's one workspace, and the next call
 * overwrites it: calls enqueued on the same stream are ordered, but calls
 * that may overlap on one GPU (different streams, or host threads racing on
 * one stream) race on the tables and must be serialised by the caller.
 * The tables are copied from pageable host memory (hipMemcpyAsync), so the
 * call returns once they are consumed; it is not meant for HIP graph capture.
 * Returns as apsp_solve_batched_ex, or APSP_ERR_UNSUPPORTED.
 */
#define APSP_NOALLOC_WORKSPACE_BYTES (8 << 20)
int32_t apsp_solve_batched_noalloc(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                   int32_t count, int32_t dtype, void *stream);

/*
 * Reusable batched plans.  apsp_batched_plan_create checks the arguments as
 * apsp_solve_batched_ex does, builds the descriptor and work-item tables on
 * the host, copies them into library-owned device memory (hipMalloc) and
 * waits for the copy on `stream`.  apsp_batched_plan_run enqueues the solve
 * of all the plan's graphs on `stream` and allocates nothing, so it may be
 * captured in a HIP graph; it may be called any number of times, for any
 * matrices now stored at the plan's pointers.  apsp_batched_plan_destroy
 * frees the tables (hipFree, which waits for the device); the caller must
 * not destroy a plan whose runs are still pending on another stream.
 * apsp_batched_plan_info writes {launches, work items, tile updates}.
 * Working copies: a graph whose rows are not 16-byte aligned (ld not a
 * multiple of 4, or a pointer off 16 bytes) would take the kernels'
 * word-by-word load path (the 4096-graph batch of n <= 512: 4.77 ms with
 * contiguous rows in place, 4.49 ms on working copies, 3.76 ms with rows
 * rounded up to 4 by the caller).  Plans and
 * the one-shot calls give each such graph a working copy of n x (n rounded
 * up to 4) words (plans: hipMalloc at creation, freed with the plan;
 * one-shot calls: hipMallocAsync, freed stream-ordered), which every run
 * fills first and copies back last; the results are the same bits.  The
 * copies are off when apsp_set_aligned_copy_min_n is above
 * APSP_BATCHED_MAX_N, and skipped when they cannot be allocated;
 * apsp_solve_batched_noalloc makes none.
 * The plan keeps the matrix pointers, not the matrices: the caller keeps
 * them allocated while the plan is used.
 */
typedef struct apsp_batch_plan apsp_batch_plan;
int32_t apsp_batched_plan_create(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                 int32_t count, int32_t dtype, void *stream,
                                 apsp_batch_plan **plan);
int32_t apsp_batched_plan_run(const apsp_batch_plan *plan, void *stream);
int32_t apsp_batched_plan_info(const apsp_batch_plan *plan, int64_t *info);
int32_t apsp_batched_plan_destroy(apsp_batch_plan *plan);

/*
 * apsp_batched_plan_create_tiled -- as apsp_batched_plan_create with the
 * round width forced: tile 64 or 128 for every graph, 0 for the batched
 * tuning table's width per graph (what apsp_batched_plan_create does).
 * Any other tile is APSP_ERR_INVALID_VALUE.  Either width is the blocked
 * method of Sec. 4.4/4.5 (Algorithms 3 and 4) with that block size.
 */
int32_t apsp_batched_plan_create_tiled(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                       int32_t count, int32_t dtype, int32_t tile, void *stream,
                                       apsp_batch_plan **plan);

/*
 * Batched tuning table.  The batched path picks each graph's round width
 * (64 or 128) from a per-device table of APSP_TUNE_BUCKETS size buckets:
 * bucket b < 8 holds n in (64b, 64b + 64], bucket 8 every n > 512.  Until a
 * device is tuned or its table is set, every bucket is 128.  Plans take the
 * widths when they are created.
 *   apsp_batched_tuning_get / _set  read / replace the current device's
 *       table (count must be APSP_TUNE_BUCKETS; set accepts 64 and 128 only
 *       and checks every entry before changing any).
 *   apsp_batched_autotune  times both widths on the current device, bucket
 *       by bucket, on a synthetic batch of batch_elems matrix elements
 *       (2^20 <= batch_elems <= 2^30; graphs of the bucket's largest n, 1024
 *       for bucket 8, back to back) and keeps 64 where it is at least 3%
 *       faster.  It allocates batch_elems * 4 bytes (hipMalloc), runs on
 *       `stream` and waits for it; the table is updated when every bucket
 *       has been timed.  table (nullable) receives the widths, ms (nullable,
 *       2 * APSP_TUNE_BUCKETS doubles) the milliseconds per run of the
 *       128-wide and the 64-wide plan of each bucket.
 * They return APSP_ERR_INVALID_VALUE for bad arguments and APSP_ERR_DEVICE
 * when there is no current device.
 */
/*
 * apsp_batched_autotune_batch -- tune the table for a given batch: the
 * graphs (arguments as apsp_batched_plan_create; count >= 1 and at least
 * one non-empty graph) are copied twice into library-owned memory
 * (hipMalloc, 2 x 4 x sum n_g * roundup(n_g, 4) bytes, freed on return), and
 * the copies are solved under greedy choices: every bucket 128 first, then
 * each bucket in the batch, in decreasing order of its share of sum n^3, is
 * switched to 64 and kept there if the whole batch solves at least 3%
 * faster (each timing is the best of five solves from the pristine copy).
 * The caller's matrices are only read.  Runs on `stream` and waits for it;
 * stores the result in the current device's table.  table (nullable)
 * receives the widths, ms (nullable, 2 doubles) the milliseconds per solve
 * with every bucket 128 and with the chosen table.
 */
int32_t apsp_batched_autotune_batch(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                    int32_t count, int32_t dtype, void *stream, int32_t *table,
                                    double *ms);

#define APSP_TUNE_BUCKETS 9
int32_t apsp_batched_tuning_get(int32_t *table, int32_t count);
int32_t apsp_batched_tuning_set(const int32_t *table, int32_t count);
int32_t apsp_batched_autotune(int32_t dtype, int64_t batch_elems, void *stream, int32_t *table,
                              double *ms);

/* Round width (64 or 128) the batched path uses for a graph of n vertices on
 * the current device, from the tuning table (128 without a device); 0 for a
 * bad dtype. */
int32_t apsp_batched_round_width(int64_t n, int32_t dtype);

/*
 * apsp_minplus -- min-plus product (Table 1: MatProd; with accumulate,
 * MinPlus = MatProd followed by MatMin):
 *   accumulate == 0:  C = A (x) B,          C_ij = min_k A_ik + B_kj
 *   accumulate != 0:  C = min(C, A (x) B)
 * C is m x n, A is m x k, B is k x n, all row-major device matrices of one
 * dtype with leading dimensions ldc >= n, lda >= k, ldb >= n.  k >= 1 (k == 0
 * is APSP_ERR_INVALID_VALUE); m == 0 or n == 0 is a no-op.  C must not
 * overlap A or B (checked on the address ranges; APSP_ERR_INVALID_VALUE).
 * Entries follow the matrix format above ("no edge" = 2^30 / +inf, values
 * >= 0); int32 sums of two entries <= 2^30 cannot wrap (computed as uint32).
 * Asynchronous on `stream`; allocates nothing.
 */
int32_t apsp_minplus(void *C, int64_t ldc, const void *A, int64_t lda, const void *B, int64_t ldb,
                     int64_t m, int64_t n, int64_t k, int32_t dtype, int32_t accumulate,
                     void *stream);

/*
 * apsp_solve_squaring -- APSP by repeated min-plus squaring (Sec. 4.2,
 * Algorithm 1): after input normalisation, X <- X (x) X is applied
 * apsp_squarings(n) = ceil(log2(n - 1)) times (n >= 3; 0 otherwise), which
 * covers every path of up to n - 1 edges.  `work` is a caller-provided
 * n x n device buffer (leading dimension ldw >= n) that must not overlap
 * `dist`; the result ends in `dist`.  Does ceil(log2(n-1)) times the work of
 * apsp_solve; int32 results are identical to it, fp32 results differ in
 * summation order only.  Asynchronous; allocates nothing.
 */
int32_t apsp_solve_squaring(void *dist, int64_t n, int64_t ld, int32_t dtype, void *work,
                            int64_t ldw, void *stream);
int32_t apsp_squarings(int64_t n);

/*
 * apsp_validate -- check the input domain (Sec. 3: non-negative weights, no
 * NaN) of an n x n matrix.  Synchronous: waits on `stream` for its own result.
 * Returns APSP_OK when every entry is >= 0 (and not NaN), APSP_ERR_BAD_INPUT
 * otherwise, or an argument / device error.  The diagonal is checked too.
 */
int32_t apsp_validate(const void *dist, int64_t n, int64_t ld, int32_t dtype, void *stream);

/* Static description of a status code (never NULL). */
const char *apsp_status_string(int32_t status);

/* The HIP call that made the calling thread's most recent call fail with
 * APSP_ERR_DEVICE or APSP_ERR_NO_MEMORY, with its error name and code
 * (empty string if none; never NULL). */
const char *apsp_last_error(void);

/* Library version string, e.g. "apsp-mi355x 0.1.0 gfx950". */
const char *apsp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* APSP_H_ */

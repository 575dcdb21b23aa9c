// Round scheduler of the single-graph solver: enqueues the phases of the
// blocked method (arXiv:1902.04446, Sec. 4.4/4.5, Algorithms 3 and 4) with a
// one-round lookahead over the library's own streams of the caller's stream
// (a chain stream S, which starts after the caller's earlier work and which
// the caller's stream waits for at the end, and band streams H).
//
// The paper's rounds are strictly ordered: phase 1 of round r+1 needs the
// diagonal block that phase 3 of round r produced.  Only the tiles in block
// row and block column r+1 are needed that early, so phase 3 of round r is
// split in two tile sets:
//
//   A(r) = phase-3 tiles in block row/column r+1      (kNext, 2q-3 tiles)
//   B(r) = every other phase-3 tile                     (kRest, (q-2)^2 tiles)
//
// and the chain stream S runs the short critical chain
//   P2(r) -> [wait B(r-1)] -> A(r) -> P2(r+1) -> [wait B(r)] -> A(r+1) -> ...
// while a band stream H runs B(r) as soon as P2(r) is done.  (Below the
// lookahead's round count everything runs on the caller's stream.)  Phase 1 of
// round r+1 is fused into A(r): the workgroup that produces diagonal block
// r+1 closes it in registers before storing it, so no single-workgroup
// kernel has to find room on a GPU filled by B(r).  B(r) overlaps A(r) and
// phase 2 of round r+1.  The sets are disjoint and each
// reads only data no concurrently running kernel writes:
//   * B(r) reads panels (r, J), (I, r) with I, J outside {r, r+1} and writes
//     tiles outside rows/columns r and r+1;
//   * P1(r+1) and P2(r+1) write only row/column r+1 tiles (A(r)'s outputs)
//     and read the diagonal block r+1; none of these is touched by B(r);
//   * A(r+1) rewrites row/column r+2 tiles, which B(r) wrote, so S waits
//     for B(r) first.
// B(r) itself runs as bands of block rows on separate band streams; band g
// of round r+1 follows band g of round r on its stream and reads only the
// panels of round r+1 and its own tiles, so it does not wait for the other
// bands of B(r), except the band holding block row r: that row was the row
// panel all bands of B(r) read, and round r+1 overwrites it.
// The last round has no round r+1: its phase 3 runs whole on S after B(r-1).
// The result is the same as running the three phases in order, bit for bit:
// every tile sees the same operands in the same round.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "apsp_common.h"

namespace apsp {

namespace {

// B(r) is split into kBands bands of block rows, each on its own helper
// stream: band g of round r+1 follows band g of round r and needs nothing
// else of B(r), so one band's launch boundary overlaps the other band's work
// instead of draining the GPU once per round.
// Measured: three bands (with the chain stream, four library streams on the
// four hardware queues) lose to two: 121 against 117 ms at n = 16384, 17.5
// against 16.7 ms at n = 8192.
#ifndef APSP_BANDS
#define APSP_BANDS 2
#endif
constexpr int kBands = APSP_BANDS;
// Below this many rounds a band launch is too short for the overlap to pay
// for the extra launch and event per round; B(r) then runs as one launch.
#ifndef APSP_MIN_BAND_ROUNDS
#define APSP_MIN_BAND_ROUNDS 64
#endif
constexpr int64_t kMinBandRounds = APSP_MIN_BAND_ROUNDS;
// Rounds of 64 from which the one-round lookahead is used.  Below it each
// round is phase 2 then the whole phase 3 (with the next closure fused) on the
// caller's stream: measured, the cross-stream events of the lookahead cost
// more than its overlap up to 48 rounds (n = 2048: 1.05 ms without, 1.24 ms
// with; n = 3072: 1.94 / 2.01), break even at 64 and win from 80 (n = 5120:
// 5.89 / 5.63 ms).
#ifndef APSP_W64_LOOKAHEAD_ROUNDS
#define APSP_W64_LOOKAHEAD_ROUNDS 64
#endif
constexpr int64_t kW64LookaheadRounds = APSP_W64_LOOKAHEAD_ROUNDS;
// From this many rounds on, phase 3 runs in round pairs (apsp_pair.hip):
// one pass with k over two blocks reads and writes each tile once per two
// rounds.  Below it the pair's longer chain of launches on the caller's
// stream is not hidden behind the rest set: measured, pairs lose 6% at 64
// rounds and win 2% at 72, 7% at 128.  Settable per process
// (apsp_set_round_pair_threshold).
constexpr int64_t kDefaultPairRounds = 72;
// int32 solves held as fp32 bits (kI32AsF32): from this many rounds of the
// matrix and of the call (the two conversion passes then cost well under
// what the direct-staged fp32 kernels gain).
constexpr int64_t kConvMinRounds = 64;
constexpr int64_t kConvMinCallRounds = 16;
std::atomic<int64_t> g_pair_rounds{kDefaultPairRounds};
// Matrices of at most this many vertices run rounds of width 64
// (apsp_small.hip): below it a solve is bound by the chain of dependent
// launches, which 64-wide rounds shorten.  Measured (fp32 Swiss-roll kNN,
// width 64 / 128): n = 256 0.13 / 0.26 ms, 1024 0.47 / 1.06, 4096 3.45 /
// 4.59, 5120 5.63 / 5.91, 6144 9.34 / 8.41.  Settable per process
// (apsp_set_width64_max_n).
constexpr int64_t kDefaultWidth64MaxN = 5120;
std::atomic<int64_t> g_w64_max_n{kDefaultWidth64MaxN};

struct Helper {
    // The solve's own streams: `chain` runs what the caller's stream would
    // (it starts after the caller's earlier work and the caller waits for
    // it), side[g] run the bands.  They are created together, one after the
    // other: HIP deals streams to its hardware queues (4 by default) in
    // creation order, so the three land on three different queues and the
    // bands overlap the chain whatever queue the caller's stream is on.
    hipStream_t chain = nullptr;
    hipStream_t side[kBands] = {};
    hipEvent_t enter = nullptr, leave = nullptr;  // caller -> chain, chain -> caller
    hipEvent_t p2_done = nullptr;             // recorded on S after P2(r)
    hipEvent_t rest_done[kBands] = {};        // recorded on H_g after band g of B(r)
    uint32_t *word = nullptr;                 // int32: largest finite entry of the matrix
    PairCopies copies;                        // round pairs: copies of round r+1's panels
    void *copies_buf = nullptr;
    size_t copies_bytes = 0;
    std::mutex mu;                            // one solve enqueues on these at a time
};

// Bytes of the round-pair copies for an n-vertex matrix: 3 block-row copies
// and 5 transposed block-column copies, each 128 x 128 q words.
size_t pair_copies_bytes(int64_t n) {
    const size_t ldc = (size_t)num_rounds(n) * kRoundB;
    return (size_t)(kPairRowSlots + 5) * kRoundB * ldc * sizeof(uint32_t);
}

// Point h->copies at their slots sized for n, growing the buffer if needed
// (growing synchronises `s` and the helper streams: solves still running on
// them may read the old buffer).  False when the memory is not there (the
// caller then runs single rounds).
bool ensure_copies(Helper *h, int64_t n, hipStream_t s) {
    const int64_t ldc = num_rounds(n) * kRoundB;
    const size_t slot_elems = (size_t)kRoundB * (size_t)ldc;
    const size_t need = pair_copies_bytes(n);
    if (h->copies_bytes < need) {
        if (h->copies_buf) {
            // earlier solves on these streams may still read the old buffer
            if (hipStreamSynchronize(s) != hipSuccess) return false;
            if (h->chain && hipStreamSynchronize(h->chain) != hipSuccess) return false;
            for (hipStream_t x : h->side)
                if (hipStreamSynchronize(x) != hipSuccess) return false;
            (void)hipFree(h->copies_buf);
            h->copies_buf = nullptr;
            h->copies_bytes = 0;
        }
        if (hipMalloc(&h->copies_buf, need) != hipSuccess) {
            (void)hipGetLastError();
            h->copies_buf = nullptr;
            return false;
        }
        h->copies_bytes = need;
    }
    uint32_t *base = static_cast<uint32_t *>(h->copies_buf);
    for (int k = 0; k < kPairRowSlots; ++k) h->copies.row[k] = base + k * slot_elems;
    for (int k = 0; k < 5; ++k) h->copies.colT[k] = base + (kPairRowSlots + k) * slot_elems;
    h->copies.ld = ldc;
    return true;
}



std::mutex g_map_mu;
std::map<std::pair<int, hipStream_t>, Helper *> g_helpers;

// Helper stream + events for (current device, caller stream), created once.
Helper *helper_for(hipStream_t s, hipError_t *err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        note_error("hipGetDevice", e);
        *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_map_mu);
    auto key = std::make_pair(dev, s);
    auto it = g_helpers.find(key);
    if (it != g_helpers.end()) return it->second;
    Helper *h = new Helper();
    const char *what = "hipStreamCreateWithFlags";
    e = hipStreamCreateWithFlags(&h->chain, hipStreamNonBlocking);
    for (int g = 0; g < kBands && e == hipSuccess; ++g)
        e = hipStreamCreateWithFlags(&h->side[g], hipStreamNonBlocking);
    if (e == hipSuccess) {
        what = "hipEventCreateWithFlags";
        e = hipEventCreateWithFlags(&h->p2_done, hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->enter, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->leave, hipEventDisableTiming);
    for (int g = 0; g < kBands && e == hipSuccess; ++g)
        e = hipEventCreateWithFlags(&h->rest_done[g], hipEventDisableTiming);
    if (e == hipSuccess) {
        what = "hipMalloc";
        e = hipMalloc(reinterpret_cast<void **>(&h->word), 256);
    }
    if (e != hipSuccess) {
        note_error(what, e);
        *err = e;
        delete h;  // leaks a partially created stream/event only on a failing device
        return nullptr;
    }
    g_helpers[key] = h;
    return h;
}

// Destroy a helper's streams and events and free its device memory (its
// work must have finished).
void destroy_helper(Helper *h) {
    if (h->chain) (void)hipStreamDestroy(h->chain);
    for (hipStream_t x : h->side)
        if (x) (void)hipStreamDestroy(x);
    if (h->enter) (void)hipEventDestroy(h->enter);
    if (h->leave) (void)hipEventDestroy(h->leave);
    if (h->p2_done) (void)hipEventDestroy(h->p2_done);
    for (hipEvent_t e : h->rest_done)
        if (e) (void)hipEventDestroy(e);
    if (h->word) (void)hipFree(h->word);
    if (h->copies_buf) (void)hipFree(h->copies_buf);
    delete h;
}

// Whether a full solve of an n-vertex matrix uses the one-round lookahead,
// and whether it runs round pairs (at the current thresholds).
bool uses_lookahead(int64_t n) {
    const int b = round_width(n);
    const int64_t q = (n + b - 1) / b;
    return q >= (b != kRoundB ? kW64LookaheadRounds : 3);
}

bool uses_pairs(int64_t n) {
    const int b = round_width(n);
    const int64_t q = (n + b - 1) / b;
    return b == kRoundB && uses_lookahead(n) && q >= g_pair_rounds.load() && q >= 2;
}

// Whether a full solve of an fp32 matrix of n vertices (or an int32 one held
// as fp32 bits, from kConvMinRounds rounds) runs single rounds of 128 with
// the direct-staged rest set (which needs the transposed column copies),
// given 16-byte aligned rows.
bool uses_direct_single(int64_t n, int dtype) {
    return (dtype == 1 || (dtype == 0 && (n + kRoundB - 1) / kRoundB >= kConvMinRounds)) &&
           n % kRoundB == 0 && round_width(n) == kRoundB && uses_lookahead(n) &&
           !uses_pairs(n);
}

// Timing events of one profiled solve.
struct Timer {
    std::vector<hipEvent_t> ev;
    bool ok = true;
    hipEvent_t make() {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            ok = false;
            return nullptr;
        }
        ev.push_back(e);
        return e;
    }
    ~Timer() {
        for (auto e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

double elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    return (a && b && hipEventElapsedTime(&ms, a, b) == hipSuccess) ? (double)ms : 0.0;
}

}  // namespace

int64_t stream_state_bytes(int64_t n, int dtype) {
    if (n <= 0 || !(uses_lookahead(n) || dtype == 0)) return 0;
    return 256 + (uses_pairs(n) || uses_direct_single(n, dtype) ? (int64_t)pair_copies_bytes(n)
                                                                 : 0);
}

int64_t stream_state_count() {
    std::lock_guard<std::mutex> lock(g_map_mu);
    return (int64_t)g_helpers.size();
}

hipError_t side_resources(hipStream_t s, int64_t n, SideResources *out,
                          std::unique_lock<std::mutex> *lock) {
    hipError_t err = hipSuccess;
    Helper *h = helper_for(s, &err);
    if (!h) return err;
    std::unique_lock<std::mutex> lk(h->mu);
    if (!ensure_copies(h, n, s)) {
        note_message("the symmetric solve's row-panel copies could not be allocated");
        return hipErrorOutOfMemory;
    }
    out->chain = h->chain;
    out->enter = h->enter;
    out->leave = h->leave;
    out->side = h->side[0];
    out->p2_done = h->p2_done;
    out->rest_done = h->rest_done[0];
    out->slot[0] = h->copies.row[0];
    out->slot[1] = h->copies.row[1];
    out->ld = h->copies.ld;
    *lock = std::move(lk);
    return hipSuccess;
}

hipError_t release_stream_state(hipStream_t s) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        note_error("hipGetDevice", e);
        return e;
    }
    const auto key = std::make_pair(dev, s);
    Helper *h = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_map_mu);
        auto it = g_helpers.find(key);
        if (it == g_helpers.end()) return hipSuccess;
        h = it->second;
    }
    {
        // no solve is enqueuing on these streams while we wait for them
        std::lock_guard<std::mutex> lock(h->mu);
        // kernels on `s` read the word and the copies; the helper streams'
        // kernels too
        e = hipStreamSynchronize(s);
        if (e == hipSuccess) e = hipStreamSynchronize(h->chain);
        for (hipStream_t x : h->side)
            if (e == hipSuccess) e = hipStreamSynchronize(x);
        if (e != hipSuccess) {
            note_error("hipStreamSynchronize (releasing a stream's state)", e);
            return e;
        }
        std::lock_guard<std::mutex> lock2(g_map_mu);
        g_helpers.erase(key);
    }
    destroy_helper(h);
    return hipSuccess;
}

hipError_t run_rounds(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r0, int64_t r1,
                      bool prologue, hipStream_t caller, PhaseTimes *times) {
    hipStream_t s = caller;  // S: the caller's stream, or the helper's chain stream
    // Round width: 64 for small matrices (apsp_small.hip), else 128.
    const int b = round_width(n);
    const bool w64 = b != kRoundB;
    const int64_t q = (n + b - 1) / b;
    if (r1 > q) r1 = q;
    if (times)
        for (double &m : times->ms) m = 0.0;
    if (n <= 0 || r0 >= r1) return hipSuccess;

    // Lookahead needs a round r+1 with a non-empty rest set; for a few
    // rounds of 64 the rest set is a handful of tiles and the cross-stream
    // events cost more than the overlap gains.
    const bool lookahead = uses_lookahead(n);
    const int bands = q >= kMinBandRounds ? kBands : 1;
    hipError_t herr = hipSuccess;
    Helper *h = (lookahead || dtype == 0) ? helper_for(s, &herr) : nullptr;
    if ((lookahead || dtype == 0) && !h) return herr;
    // int32: the tiles take the fp32 pipe when this matrix allows it exactly
    const uint32_t *wmax = dtype == 0 ? h->word : nullptr;
    // int32 with rounds of 128 on aligned full tiles, from 64 rounds and for
    // a call of 16 or more: the matrix is held as the fp32 bits OpI32F
    // computes on for the call (converted in after the weight scan when that
    // scan allows the fp32 pipe, back at the end), so the fp32 kernels, with
    // their direct staging, run it (kI32AsF32).
    const bool conv = dtype == 0 && !w64 && lookahead && q >= kConvMinRounds &&
                      r1 - r0 >= kConvMinCallRounds && pair_rest_direct(D, n, ld, kI32AsF32);
    const int dt = conv ? kI32AsF32 : dtype;  // the dtype the round kernels take
    std::unique_lock<std::mutex> lock;
    if (h) lock = std::unique_lock<std::mutex>(h->mu);
    // Pairs run on the helper streams, which exist from 3 rounds on (below
    // that a pair has no rest set anyway), whatever the threshold.
    const bool pairs = !w64 && lookahead && q >= g_pair_rounds.load() && r1 - r0 >= 2 &&
                       ensure_copies(h, n, s);
    // Single rounds of 128 on an aligned fp32 matrix: phase 2 also writes its
    // block column transposed (two slots, rounds alternating), and round r's
    // phase 3 reads it with both operands staged straight into LDS.  The next
    // writer of a slot is phase 2 of round r+2, which follows the wait for
    // round r's rest set on S.
    const bool direct1 = !w64 && lookahead && !pairs && pair_rest_direct(D, n, ld, dt) &&
                         ensure_copies(h, n, s);
    if (lookahead) {
        // S = the chain stream, after the caller's earlier work
        hipError_t e = hipEventRecord(h->enter, caller);
        if (e == hipSuccess) e = hipStreamWaitEvent(h->chain, h->enter, 0);
        if (e != hipSuccess) {
            note_error("entering the solve's streams", e);
            return e;
        }
        s = h->chain;
    }
    // the phase launches at this width
    auto phase1 = [&](int64_t r) {
        return w64 ? launch_phase1_64(D, n, ld, dtype, r, s)
                   : launch_phase1(D, n, ld, dt, r, s, wmax);
    };
    auto tile_set = [&](int64_t r, int set, bool close_next) {
        return w64 ? launch_tile_set64(D, n, ld, dtype, r, set, s, close_next, wmax, 0, q)
                   : launch_tile_set(D, n, ld, dt, r, set, s, close_next, wmax);
    };
    auto rest_rows = [&](int64_t r, int64_t lo, int64_t hi, hipStream_t st) {
        return w64 ? launch_tile_set64(D, n, ld, dtype, r, kRest, st, false, wmax, lo, hi)
                   : launch_rest_rows(D, n, ld, dt, r, lo, hi, st, wmax);
    };

    // Timing: spans of enqueued work on a stream, by category (the PhaseTimes
    // index: 1 phase 1, 2 phase 2, 7 phase 3 on the caller's stream, 5 the
    // bands of the rest set), from events created before anything is enqueued.
    Timer tm;
    struct Span {
        int cat;
        hipEvent_t b, e;
    };
    std::vector<Span> spans;
    std::vector<hipEvent_t> pool;
    size_t pool_next = 0;
    hipEvent_t t_begin = nullptr, t_pro = nullptr, t_end = nullptr;
    auto rec = [&](hipEvent_t e, hipStream_t st) {
        if (e && hipEventRecord(e, st) != hipSuccess) tm.ok = false;
    };
    auto open = [&](int cat, hipStream_t st) -> size_t {
        if (!times || pool_next + 2 > pool.size()) return SIZE_MAX;
        spans.push_back(Span{cat, pool[pool_next], pool[pool_next + 1]});
        pool_next += 2;
        rec(spans.back().b, st);
        return spans.size() - 1;
    };
    auto close = [&](size_t i, hipStream_t st) {
        if (i != SIZE_MAX) rec(spans[i].e, st);
    };
    if (times) {
        t_begin = tm.make();
        t_pro = tm.make();
        t_end = tm.make();
        const size_t per_round = 2 * (4 + kBands);
        pool.resize((size_t)(r1 - r0 + 2) * per_round);
        for (auto &e : pool) e = tm.make();
        if (!tm.ok) return hipErrorOutOfMemory;
        rec(t_begin, s);
    }

    hipError_t err = hipSuccess;
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && err == hipSuccess) {
            err = e;
            note_error("kernel launch or stream call", e);
        }
    };
    if (prologue) chk(launch_prologue(D, n, ld, dtype, s));
    if (wmax) chk(launch_wmax(D, n, ld, h->word, s));
    if (conv) chk(launch_conv_i32(D, n, ld, h->word, true, s));
    if (times) rec(t_pro, s);

    bool rest_pending = false;
    bool diag_closed = false;  // phase 1 of round r already ran inside an earlier launch
    int64_t rest_launches = 0;
    auto wait_rest = [&](hipStream_t st) {
        if (rest_pending)
            for (int g = 0; g < bands; ++g) chk(hipStreamWaitEvent(st, h->rest_done[g], 0));
    };
    auto band_range = [&](int g, int64_t &lo, int64_t &hi) {
        lo = q * g / bands;  // band g: block rows [q g / bands, q (g+1) / bands)
        hi = q * (g + 1) / bands;
    };
    // A round's phase 1 + 2 on S (phase 1 unless an earlier launch fused it).
    auto phases12 = [&](int64_t r) {
        size_t sp = open(1, s);
        if (!diag_closed) chk(phase1(r));
        close(sp, s);
        diag_closed = false;
        sp = open(2, s);
        if (direct1)
            chk(launch_pair_panels(D, n, ld, dt, r, h->copies, -1, (int)(r & 1), s, wmax));
        else
            chk(tile_set(r, kPanels, false));
        close(sp, s);
    };

    if (pairs) {
        // Round pairs (r, r+1), see apsp_pair.hip.  On S: phases 1-2 of
        // round r (its block column copied transposed to slot first), round
        // r's phase 3 on block row/column r+1 with the closure of block r+1,
        // phase 2 of round r+1 (its panels copied to slot `slot`); then,
        // after the previous pair's rest set, the pair pass on block
        // rows/columns r+2, r+3 (closing block r+2) and the deferred updates
        // of tiles (x, r), (r, x).  The rest set runs in bands on the helper
        // streams as soon as phase 2 of round r+1 is done.  A band that
        // holds block row prev or prev+1 (the previous pair) waits for every
        // band of the previous pair: all of them read those rows.
        // Copy slots: `slot` cycles over three, so the previous pair's copies
        // (read by this pair's deferred updates) are not overwritten before
        // S has waited for this pair's bands; `first` alternates between two,
        // its only readers being the pair's own bands, which S waits for
        // before the pair after next writes it again.
        int64_t prev = -1;
        int prev_slot = 0, slot = 0, first = kPairFirstSlot0;
        int64_t r = r0;
        while (r < r1 && err == hipSuccess) {
            if (r + 1 >= r1) {  // the call's last round alone
                wait_rest(s);
                rest_pending = false;
                if (prev >= 0) {
                    const size_t sp = open(7, s);
                    chk(launch_pair_fix(D, n, ld, dt, prev, true, s, wmax));
                    close(sp, s);
                    prev = -1;
                }
                phases12(r);
                const size_t sp = open(7, s);
                chk(tile_set(r, kAll, false));
                close(sp, s);
                ++r;
                break;
            }
            const int nx = pair_next_blocks(n, r);
            {  // phases 1-2 of round r, its block column copied transposed
                size_t sp1 = open(1, s);
                if (!diag_closed) chk(launch_phase1(D, n, ld, dt, r, s, wmax));
                close(sp1, s);
                diag_closed = false;
                sp1 = open(2, s);
                chk(launch_pair_panels(D, n, ld, dt, r, h->copies, -1, first, s, wmax));
                close(sp1, s);
            }
            size_t sp = open(7, s);
            chk(launch_pair_round_next(D, n, ld, dt, r, h->copies, first, s, wmax));
            close(sp, s);
            sp = open(2, s);
            chk(launch_pair_panels(D, n, ld, dt, r + 1, h->copies, slot, slot, s, wmax));
            close(sp, s);
            chk(hipEventRecord(h->p2_done, s));
            wait_rest(s);
            const bool close_next = nx > 0 && r + 2 < r1;
            sp = open(7, s);
            if (nx > 0) {
                chk(launch_pair_next(D, n, ld, dt, r, close_next, prev, h->copies, prev_slot,
                                     first, slot, s, wmax));
                chk(launch_pair_fix(D, n, ld, dt, r, false, s, wmax));
            }
            close(sp, s);
            diag_closed = close_next;
            for (int g = 0; g < bands; ++g) {
                int64_t lo, hi;
                band_range(g, lo, hi);
                if (rest_pending && prev >= 0 &&
                    ((prev >= lo && prev < hi) || (prev + 1 >= lo && prev + 1 < hi)))
                    for (int o = 0; o < bands; ++o)
                        if (o != g) chk(hipStreamWaitEvent(h->side[g], h->rest_done[o], 0));
            }
            for (int g = 0; g < bands; ++g) {
                int64_t lo, hi;
                band_range(g, lo, hi);
                chk(hipStreamWaitEvent(h->side[g], h->p2_done, 0));
                const size_t b = open(5, h->side[g]);
                chk(launch_pair_rest(D, n, ld, dt, r, lo, hi, prev, h->copies, prev_slot,
                                     first, slot, h->side[g], wmax));
                close(b, h->side[g]);
                chk(hipEventRecord(h->rest_done[g], h->side[g]));
            }
            rest_pending = true;
            ++rest_launches;
            prev = r;
            prev_slot = slot;
            slot = (slot + 1) % kPairRowSlots;
            first = first == kPairFirstSlot0 ? kPairFirstSlot0 + 1 : kPairFirstSlot0;
            r += 2;
        }
        wait_rest(s);
        if (prev >= 0 && err == hipSuccess) {
            const size_t sp = open(7, s);
            chk(launch_pair_fix(D, n, ld, dt, prev, true, s, wmax));
            close(sp, s);
        }
    } else {
        for (int64_t r = r0; r < r1 && err == hipSuccess; ++r) {
            phases12(r);
            if (lookahead && r + 1 < q) {
                // Fuse phase 1 of round r+1 into A(r) unless this call stops
                // after round r: a solve split over calls leaves exactly the
                // state of Floyd-Warshall after its last round's pivots.
                const bool fuse = r + 1 < r1;
                chk(hipEventRecord(h->p2_done, s));
                wait_rest(s);
                size_t sp = open(7, s);
                if (direct1 && fuse)  // (the direct form always closes block r+1)
                    chk(launch_pair_round_next(D, n, ld, dt, r, h->copies, (int)(r & 1), s,
                                               wmax));
                else
                    chk(tile_set(r, kNext, fuse));
                close(sp, s);
                diag_closed = fuse;
                for (int g = 0; g < bands; ++g) {
                    int64_t lo, hi;
                    band_range(g, lo, hi);
                    // Block row r-1 was the row panel every band of B(r-1)
                    // read; the band that now updates it waits for all of
                    // B(r-1).  (The events still hold round r-1: this round
                    // records them below.)
                    if (rest_pending && r - 1 >= lo && r - 1 < hi)
                        for (int o = 0; o < bands; ++o)
                            if (o != g) chk(hipStreamWaitEvent(h->side[g], h->rest_done[o], 0));
                }
                for (int g = 0; g < bands; ++g) {
                    int64_t lo, hi;
                    band_range(g, lo, hi);
                    chk(hipStreamWaitEvent(h->side[g], h->p2_done, 0));
                    const size_t b = open(5, h->side[g]);
                    if (direct1)
                        chk(launch_round_rest_direct(D, n, ld, dt, r, lo, hi, h->copies,
                                                     (int)(r & 1), h->side[g], wmax));
                    else
                        chk(rest_rows(r, lo, hi, h->side[g]));
                    close(b, h->side[g]);
                    chk(hipEventRecord(h->rest_done[g], h->side[g]));
                }
                rest_pending = true;
                ++rest_launches;
            } else {
                // whole phase 3 on S; its workgroup of diagonal block r+1
                // closes it (phase 1 of round r+1) unless the call stops here
                wait_rest(s);
                rest_pending = false;
                const bool fuse = r + 1 < r1;
                const size_t sp = open(7, s);
                chk(tile_set(r, kAll, fuse));
                close(sp, s);
                diag_closed = fuse;
            }
        }
        wait_rest(s);
    }
    if (conv && err == hipSuccess) chk(launch_conv_i32(D, n, ld, h->word, false, s));
    if (s != caller) {  // the caller's stream waits for S (which waited for every band)
        chk(hipEventRecord(h->leave, s));
        chk(hipStreamWaitEvent(caller, h->leave, 0));
    }
    if (err != hipSuccess) return err;
    if (!times) return hipSuccess;

    rec(t_end, s);
    if (!tm.ok) return hipErrorUnknown;
    if ((err = hipEventSynchronize(t_end)) != hipSuccess) return err;
    double *m = times->ms;
    m[0] = elapsed(t_begin, t_pro);
    // rest set: the time during which any band launch ran (the union of their
    // intervals; bands of consecutive rounds or pairs overlap)
    std::vector<std::pair<double, double>> bspans;
    for (const Span &sp : spans) {
        if (sp.cat == 5)
            bspans.emplace_back(elapsed(t_begin, sp.b), elapsed(t_begin, sp.e));
        else
            m[sp.cat] += elapsed(sp.b, sp.e);
    }
    std::sort(bspans.begin(), bspans.end());
    double cover = 0.0, lo = 0.0, hi = -1.0;
    for (const auto &sp : bspans) {
        if (sp.first > hi) {
            if (hi > lo) cover += hi - lo;
            lo = sp.first;
            hi = sp.second;
        } else if (sp.second > hi) {
            hi = sp.second;
        }
    }
    if (hi > lo) cover += hi - lo;
    m[5] = cover;
    m[6] = (double)rest_launches;
    m[3] = m[7] + cover;
    m[4] = elapsed(t_begin, t_end);
    return hipSuccess;
}

int64_t set_pair_rounds(int64_t rounds) { return g_pair_rounds.exchange(rounds); }

int round_width(int64_t n) { return n <= g_w64_max_n.load() ? 64 : kRoundB; }

int64_t set_width64_max_n(int64_t n) { return g_w64_max_n.exchange(n); }

}  // namespace apsp

// Round scheduler of the single-graph solver: enqueues the phases of the
// blocked method (arXiv:1902.04446, Sec. 4.4/4.5, Algorithms 3 and 4) with a
// one-round lookahead over two HIP streams.
//
// The paper's rounds are strictly ordered: phase 1 of round r+1 needs the
// diagonal block that phase 3 of round r produced.  Only the tiles in block
// row and block column r+1 are needed that early, so phase 3 of round r is
// split in two tile sets:
//
//   A(r) = phase-3 tiles in block row/column r+1      (kNext, 2q-3 tiles)
//   B(r) = every other phase-3 tile                     (kRest, (q-2)^2 tiles)
//
// and the caller's stream S runs the short critical chain
//   P2(r) -> [wait B(r-1)] -> A(r) -> P2(r+1) -> [wait B(r)] -> A(r+1) -> ...
// while a helper stream H runs B(r) as soon as P2(r) is done.  Phase 1 of
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
// B(r) itself runs as bands of block rows on separate helper streams; band g
// of round r+1 follows band g of round r on its stream and reads only the
// panels of round r+1 and its own tiles, so it does not wait for the other
// bands of B(r), except the band holding block row r: that row was the row
// panel all bands of B(r) read, and round r+1 overwrites it.
// The last round has no round r+1: its phase 3 runs whole on S after B(r-1).
// The result is the same as running the three phases in order, bit for bit:
// every tile sees the same operands in the same round.
#include <algorithm>
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
constexpr int kBands = 2;
// Below this many rounds a band launch is too short for the overlap to pay
// for the extra launch and event per round; B(r) then runs as one launch.
#ifndef APSP_MIN_BAND_ROUNDS
#define APSP_MIN_BAND_ROUNDS 64
#endif
constexpr int64_t kMinBandRounds = APSP_MIN_BAND_ROUNDS;

struct Helper {
    hipStream_t side[kBands] = {};
    hipEvent_t p2_done = nullptr;             // recorded on S after P2(r)
    hipEvent_t rest_done[kBands] = {};        // recorded on H_g after band g of B(r)
    uint32_t *word = nullptr;                 // int32: largest finite entry of the matrix
    std::mutex mu;                            // one solve enqueues on these at a time
};



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
    for (int g = 0; g < kBands && e == hipSuccess; ++g)
        e = hipStreamCreateWithFlags(&h->side[g], hipStreamNonBlocking);
    if (e == hipSuccess) {
        what = "hipEventCreateWithFlags";
        e = hipEventCreateWithFlags(&h->p2_done, hipEventDisableTiming);
    }
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

hipError_t run_rounds(uint32_t *D, int64_t n, int64_t ld, int dtype, int64_t r0, int64_t r1,
                      bool prologue, hipStream_t s, PhaseTimes *times) {
    const int64_t q = num_rounds(n);
    if (r1 > q) r1 = q;
    if (times)
        for (double &m : times->ms) m = 0.0;
    if (n <= 0 || r0 >= r1) return hipSuccess;

    // Lookahead needs a round r+1 with a non-empty rest set.
    const bool lookahead = q >= 3;
    const int bands = q >= kMinBandRounds ? kBands : 1;
    hipError_t herr = hipSuccess;
    Helper *h = (lookahead || dtype == 0) ? helper_for(s, &herr) : nullptr;
    if ((lookahead || dtype == 0) && !h) return herr;
    // int32: the tiles take the fp32 pipe when this matrix allows it exactly
    const uint32_t *wmax = dtype == 0 ? h->word : nullptr;
    std::unique_lock<std::mutex> lock;
    if (h) lock = std::unique_lock<std::mutex>(h->mu);

    Timer tm;
    struct RoundEv {
        hipEvent_t start, p1, p2, a0, a1, b0[kBands], b1[kBands];
    };
    std::vector<RoundEv> rev;
    hipEvent_t t_begin = nullptr, t_pro = nullptr, t_end = nullptr;
    auto rec = [&](hipEvent_t e, hipStream_t st) {
        if (e && hipEventRecord(e, st) != hipSuccess) tm.ok = false;
    };
    if (times) {
        t_begin = tm.make();
        t_pro = tm.make();
        t_end = tm.make();
        rev.resize((size_t)(r1 - r0));
        for (auto &e : rev) {
            e.start = tm.make(); e.p1 = tm.make(); e.p2 = tm.make();
            e.a0 = tm.make(); e.a1 = tm.make();
            for (int g = 0; g < kBands; ++g) {
                e.b0[g] = tm.make();
                e.b1[g] = tm.make();
            }
        }
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
    if (times) rec(t_pro, s);

    bool rest_pending = false;
    bool diag_closed = false;  // phase 1 of round r already ran inside A(r-1)
    for (int64_t r = r0; r < r1 && err == hipSuccess; ++r) {
        RoundEv *e = times ? &rev[(size_t)(r - r0)] : nullptr;
        if (e) rec(e->start, s);
        if (!diag_closed) chk(launch_phase1(D, n, ld, dtype, r, s));
        diag_closed = false;
        if (e) rec(e->p1, s);
        chk(launch_tile_set(D, n, ld, dtype, r, kPanels, s, false, wmax));
        if (e) rec(e->p2, s);
        if (lookahead && r + 1 < q) {
            // Fuse phase 1 of round r+1 into A(r) unless this call stops after
            // round r: a solve split over calls leaves exactly the state of
            // Floyd-Warshall after its last round's pivots.
            const bool fuse = r + 1 < r1;
            chk(hipEventRecord(h->p2_done, s));
            if (rest_pending)
                for (int g = 0; g < bands; ++g) chk(hipStreamWaitEvent(s, h->rest_done[g], 0));
            if (e) rec(e->a0, s);
            chk(launch_tile_set(D, n, ld, dtype, r, kNext, s, fuse, wmax));
            if (e) rec(e->a1, s);
            diag_closed = fuse;
            for (int g = 0; g < bands; ++g) {
                // band g: block rows [q g / bands, q (g+1) / bands)
                const int64_t lo = q * g / bands, hi = q * (g + 1) / bands;
                // Block row r-1 was the row panel every band of B(r-1) read;
                // the band that now updates it waits for all of B(r-1).  (The
                // events still hold round r-1: this round records them below.)
                if (rest_pending && r - 1 >= lo && r - 1 < hi)
                    for (int o = 0; o < bands; ++o)
                        if (o != g) chk(hipStreamWaitEvent(h->side[g], h->rest_done[o], 0));
            }
            for (int g = 0; g < bands; ++g) {
                const int64_t lo = q * g / bands, hi = q * (g + 1) / bands;
                chk(hipStreamWaitEvent(h->side[g], h->p2_done, 0));
                if (e) rec(e->b0[g], h->side[g]);
                chk(launch_rest_rows(D, n, ld, dtype, r, lo, hi, h->side[g], wmax));
                if (e) rec(e->b1[g], h->side[g]);
                chk(hipEventRecord(h->rest_done[g], h->side[g]));
            }
            rest_pending = true;
        } else {
            if (rest_pending)
                for (int g = 0; g < bands; ++g) chk(hipStreamWaitEvent(s, h->rest_done[g], 0));
            rest_pending = false;
            if (e) rec(e->a0, s);
            chk(launch_tile_set(D, n, ld, dtype, r, kAll, s, false, wmax));
            if (e) rec(e->a1, s);
        }
    }
    if (rest_pending)
        for (int g = 0; g < bands; ++g) chk(hipStreamWaitEvent(s, h->rest_done[g], 0));
    if (err != hipSuccess) return err;
    if (!times) return hipSuccess;

    rec(t_end, s);
    if (!tm.ok) return hipErrorUnknown;
    if ((err = hipEventSynchronize(t_end)) != hipSuccess) return err;
    double *m = times->ms;
    m[0] = elapsed(t_begin, t_pro);
    // B: the time during which any band of any round ran (the union of the
    // band launches' intervals; bands of consecutive rounds overlap)
    std::vector<std::pair<double, double>> spans;
    for (int64_t r = r0; r < r1; ++r) {
        const RoundEv &e = rev[(size_t)(r - r0)];
        m[1] += elapsed(e.start, e.p1);
        m[2] += elapsed(e.p1, e.p2);
        m[7] += elapsed(e.a0, e.a1);
        if (lookahead && r + 1 < q) {
            for (int g = 0; g < bands; ++g)
                spans.emplace_back(elapsed(t_begin, e.b0[g]), elapsed(t_begin, e.b1[g]));
            m[6] += 1.0;
        }
    }
    std::sort(spans.begin(), spans.end());
    double cover = 0.0, lo = 0.0, hi = -1.0;
    for (const auto &sp : spans) {
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
    m[3] = m[7] + cover;
    m[4] = elapsed(t_begin, t_end);
    return hipSuccess;
}

}  // namespace apsp

// Batched-solve plans: the per-graph descriptors and the per-launch work
// items of the round-synchronous batched schedule (see apsp_batched.hip),
// built on the host once and kept in device memory, so running a plan is
// nothing but kernel launches (and can be captured in a HIP graph).
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/apsp.h"
#include "apsp_common.h"

struct apsp_batch_plan {
    int dtype = 0;
    int device = 0;
    bool stream_ordered = false;  // buffers from hipMallocAsync (one-shot plans)
    apsp::BatchDesc *d_descs = nullptr;  // graphs descriptors, then (int32) wmax
    apsp::BatchItem *d_items = nullptr;
    uint32_t *d_wmax = nullptr;          // int32: largest finite weight per graph
    int32_t graphs = 0;                  // non-empty graphs
    apsp::XcdRanges scan = {};           // int32: the 128 x 128 tiles the weight scan reads
    struct Launch {
        int r;
        bool close_only;
        apsp::XcdRanges ranges;
    };
    std::vector<Launch> launches;
    int64_t items = 0;
    int64_t tiles = 0;  // tile updates (phase 2/3 items), for reporting
    // working copies of the graphs whose rows are not 16-byte aligned: the
    // descriptors point at them; a run copies them in first and back last
    uint32_t *work = nullptr;
    apsp::BatchCopy *d_copies = nullptr;  // in the table buffer
    int32_t copies = 0;
    int64_t copy_rows = 0;
};

namespace apsp {

// Build the plan's host tables.  Every graph gets a round width (64 or 128):
// `tile` forces one for all, else `table` (per size bucket) when given, else
// the device's tuning table (read once).  Launch 0 is phase 1 of round 0 for
// every graph; launches 2r+1 and 2r+2 are phases 2 and 3 of round r for every
// graph that has a round r at its own width, with the closure of diagonal
// block r+1 fused into phase 3.  int32 plans also list the 128 x 128 tiles
// of every graph for the weight scan that precedes the solve.
int32_t plan_build(apsp_batch_plan &p, void *const *ptrs, const int32_t *ns, const int64_t *lds,
                   int32_t count, int tile, const int32_t *table, std::vector<BatchDesc> &descs,
                   std::vector<BatchItem> &items) {
    descs.clear();
    items.clear();
    p.launches.clear();
    int32_t dev_table[kTuneBuckets];
    if (!tile && !table) {
        batched_tuning_snapshot(dev_table);
        table = dev_table;
    }
    for (int32_t g = 0; g < count; ++g) {
        if (ns[g] == 0) continue;
        BatchDesc d;
        d.ptr = static_cast<uint32_t *>(ptrs[g]);
        d.ld = lds ? lds[g] : (ns[g] > 1 ? ns[g] : 1);
        d.n = ns[g];
        d.tile = tile ? tile : table[batched_bucket(ns[g])];
        descs.push_back(d);
    }
    const int G = (int)descs.size();
    p.graphs = G;
    if (G == 0) return APSP_OK;
    std::vector<int> q(G);
    for (int g = 0; g < G; ++g) q[g] = (descs[g].n + descs[g].tile - 1) / descs[g].tile;

    // Balance graphs over the 8 XCDs by work (longest first, least loaded
    // XCD), so each XCD's item list of every launch is about as long.
    // (graphs by n descending, equal n in batch order: a counting sort)
    std::vector<int> order(G);
    {
        int nmax = 0;
        for (int g = 0; g < G; ++g) nmax = std::max(nmax, (int)descs[g].n);
        std::vector<int> at((size_t)nmax + 2, 0);
        for (int g = 0; g < G; ++g) ++at[(size_t)(nmax - descs[g].n) + 1];
        for (int k = 1; k <= nmax + 1; ++k) at[(size_t)k] += at[(size_t)k - 1];
        for (int g = 0; g < G; ++g) order[(size_t)at[(size_t)(nmax - descs[g].n)]++] = g;
    }
    std::vector<int> xcd(G, 0);
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // (q b)^3 per XCD, below 2^40 per graph
    int qmax = 0;
    for (int g : order) {
        const int64_t e = (int64_t)q[g] * descs[g].tile;
        int best = 0;
        for (int x = 1; x < 8; ++x) best = load[x] < load[best] ? x : best;
        xcd[g] = best;
        load[best] += e * e * e;
        qmax = std::max(qmax, q[g]);
    }
    // graphs of each width, largest first: those with a round r are a prefix
    std::vector<int> by_width[2];
    for (int g : order) by_width[descs[g].tile == 64 ? 1 : 0].push_back(g);

    // Launch 0 is phase 1 of round 0; launches 2r+1, 2r+2 are phases 2 and 3
    // of round r.  Items are written in place: first the number of items of
    // every (launch, XCD) pair, whose prefix sums give each pair's range,
    // then the items, graph by graph, at their pair's cursor.
    const int nl = 1 + 2 * qmax;
    std::vector<int64_t> cnt((size_t)nl * 8, 0);
    for (int g = 0; g < G; ++g) {
        const int64_t qg = q[g];
        int64_t *c = cnt.data() + xcd[g];
        c[0] += 1;
        if (qg > 1)
            for (int64_t r = 0; r < qg; ++r) {
                c[(2 * r + 1) * 8] += 2 * (qg - 1);
                c[(2 * r + 2) * 8] += (qg - 1) * (qg - 1);
            }
    }
    std::vector<int64_t> cur((size_t)nl * 8);
    int64_t pos = 0;
    p.launches.resize((size_t)nl);
    for (int l = 0; l < nl; ++l) {
        auto &L = p.launches[(size_t)l];
        L.r = l == 0 ? 0 : (l - 1) / 2;
        L.close_only = l == 0;
        for (int x = 0; x < 8; ++x) {
            L.ranges.offset[x] = (int32_t)pos;
            L.ranges.count[x] = (int32_t)cnt[(size_t)l * 8 + x];
            cur[(size_t)l * 8 + x] = pos;
            pos += cnt[(size_t)l * 8 + x];
        }
    }
    const int64_t launch_items = pos;
    int64_t scan_items = 0;
    if (p.dtype == APSP_I32)
        for (int g = 0; g < G; ++g) {
            const int64_t qs = (descs[g].n + kRoundB - 1) / kRoundB;
            scan_items += qs * qs;
        }
    items.resize((size_t)(launch_items + scan_items));
    BatchItem *out = items.data();
    auto put = [&](int l, int g, int I, int J) {
        BatchItem &it = out[cur[(size_t)l * 8 + xcd[g]]++];
        it.graph = g;
        it.ij = (I << 16) | J;
    };
    // Within a launch the longest items go first, where they overlap the
    // rest of the launch instead of its tail: 128-wide before 64-wide, and in
    // phase 3 the diagonal block r+1 (whose workgroup also closes it) first.
    for (int w = 0; w < 2; ++w)
        for (int g : by_width[w]) put(0, g, 0, 0);  // phase 1 of round 0, every graph
    for (int r = 0; r < qmax; ++r) {
        const int l2 = 2 * r + 1, l3 = 2 * r + 2;
        for (int w = 0; w < 2; ++w)
            for (int g : by_width[w]) {  // phase 2 of round r
                const int qg = q[g];
                if (qg <= r) break;  // and every later (smaller) graph of this width
                if (qg == 1) continue;
                for (int J = 0; J < qg; ++J)
                    if (J != r) put(l2, g, r, J);
                for (int I = 0; I < qg; ++I)
                    if (I != r) put(l2, g, I, r);
            }
        for (int w = 0; w < 2; ++w) {  // phase 3 of round r
            for (int g : by_width[w]) {
                const int qg = q[g];
                if (qg <= r) break;
                if (qg > 1 && r + 1 < qg) put(l3, g, r + 1, r + 1);
            }
            for (int g : by_width[w]) {
                const int qg = q[g];
                if (qg <= r) break;
                if (qg == 1) continue;
                for (int I = 0; I < qg; ++I) {
                    if (I == r) continue;
                    for (int J = 0; J < qg; ++J)
                        if (J != r && !(I == r + 1 && J == r + 1)) put(l3, g, I, J);
                }
            }
        }
    }
    if (p.dtype == APSP_I32) {
        // the weight scan: every 128 x 128 tile of every graph, dealt to the
        // XCDs in turn
        int64_t sc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t k = 0; k < scan_items; ++k) ++sc[k & 7];
        int64_t sp[8];
        int64_t at = launch_items;
        for (int x = 0; x < 8; ++x) {
            p.scan.offset[x] = (int32_t)at;
            p.scan.count[x] = (int32_t)sc[x];
            sp[x] = at;
            at += sc[x];
        }
        int64_t next = 0;
        for (int g = 0; g < G; ++g) {
            const int qs = (descs[g].n + kRoundB - 1) / kRoundB;
            for (int I = 0; I < qs; ++I)
                for (int J = 0; J < qs; ++J) {
                    BatchItem &it = out[sp[next++ & 7]++];
                    it.graph = g;
                    it.ij = (I << 16) | J;
                }
        }
    }
    p.items = (int64_t)items.size();
    p.tiles = 0;
    for (const auto &L : p.launches)
        if (!L.close_only)
            for (int x = 0; x < 8; ++x) p.tiles += L.ranges.count[x];
    return APSP_OK;
}

}  // namespace apsp

namespace {

bool bad_dtype(int32_t dtype) { return dtype != APSP_I32 && dtype != APSP_F32; }

int32_t check_batch(void *const *ptrs, const int32_t *ns, const int64_t *lds, int32_t count,
                    int32_t dtype) {
    if (bad_dtype(dtype) || count < 0) return APSP_ERR_INVALID_VALUE;
    if (count == 0) return APSP_OK;
    if (ptrs == nullptr || ns == nullptr) return APSP_ERR_INVALID_VALUE;
    for (int32_t g = 0; g < count; ++g) {
        const int64_t n = ns[g];
        const int64_t ld = lds ? lds[g] : (n > 1 ? n : 1);
        if (n < 0 || n > APSP_BATCHED_MAX_N) return APSP_ERR_INVALID_VALUE;
        if (ld < (n > 1 ? n : 1)) return APSP_ERR_INVALID_VALUE;
        if (n > 0 && ptrs[g] == nullptr) return APSP_ERR_INVALID_VALUE;
    }
    return APSP_OK;
}

// The device tables of a plan are one buffer: the graph descriptors, then
// (int32) one word per graph for its largest finite weight, then (16-byte
// aligned) the work items, then the working-copy entries.
struct TableLayout {
    size_t wmax_off, items_off, copies_off, total;
};

TableLayout table_layout(size_t graphs, size_t items, size_t copies, int32_t dtype) {
    TableLayout t;
    t.wmax_off = graphs * sizeof(apsp::BatchDesc);
    const size_t wb = dtype == APSP_I32 ? graphs * sizeof(uint32_t) : 0;
    t.items_off = (t.wmax_off + wb + 15) / 16 * 16;
    t.copies_off = (t.items_off + items * sizeof(apsp::BatchItem) + 15) / 16 * 16;
    t.total = t.copies_off + copies * sizeof(apsp::BatchCopy);
    return t;
}

// The tables in one host buffer, laid out as on the device (the weight words
// are left for the scan launch to fill).
void pack_tables(const std::vector<apsp::BatchDesc> &descs,
                 const std::vector<apsp::BatchItem> &items,
                 const std::vector<apsp::BatchCopy> &copies, const TableLayout &t,
                 std::vector<unsigned char> &host) {
    host.assign(t.total, 0);
    std::memcpy(host.data(), descs.data(), descs.size() * sizeof(apsp::BatchDesc));
    std::memcpy(host.data() + t.items_off, items.data(), items.size() * sizeof(apsp::BatchItem));
    if (!copies.empty())
        std::memcpy(host.data() + t.copies_off, copies.data(),
                    copies.size() * sizeof(apsp::BatchCopy));
}

void point_tables(apsp_batch_plan *p, void *base, const TableLayout &t) {
    unsigned char *b = static_cast<unsigned char *>(base);
    p->d_descs = reinterpret_cast<apsp::BatchDesc *>(b);
    p->d_wmax = p->dtype == APSP_I32 ? reinterpret_cast<uint32_t *>(b + t.wmax_off) : nullptr;
    p->d_items = reinterpret_cast<apsp::BatchItem *>(b + t.items_off);
    p->d_copies = p->copies ? reinterpret_cast<apsp::BatchCopy *>(b + t.copies_off) : nullptr;
}

void free_plan_buffers(apsp_batch_plan *p, hipStream_t s) {
    for (void *buf : {static_cast<void *>(p->d_descs), static_cast<void *>(p->work)}) {
        if (!buf) continue;
        if (p->stream_ordered)
            (void)hipFreeAsync(buf, s);
        else
            (void)hipFree(buf);
    }
    p->d_descs = nullptr;
    p->d_items = nullptr;
    p->d_wmax = nullptr;
    p->d_copies = nullptr;
    p->work = nullptr;
}

// Working copies for the graphs whose rows are not 16-byte aligned (their
// tiles would take the word-by-word load path: the 4096-graph batch with
// contiguous rows runs 4.77 ms in place, 4.49 ms on working copies, against
// 3.76 ms with rows rounded up to 4 elements by the caller): one buffer of
// n x (n rounded up to 4) words per such graph,
// the descriptors pointed at them.  Off when the working-copy threshold is
// above every batched size, and skipped (the graphs run in place) when the
// buffer cannot be allocated.
void plan_working_copies(apsp_batch_plan *p, std::vector<apsp::BatchDesc> &descs,
                         std::vector<apsp::BatchCopy> &copies, hipStream_t s) {
    copies.clear();
    if (apsp::aligned_copy_min_n() > APSP_BATCHED_MAX_N) return;
    thread_local std::vector<size_t> which;  // the descriptor of each copy
    which.clear();
    int64_t words = 0, rows = 0;
    for (size_t g = 0; g < descs.size(); ++g) {
        const apsp::BatchDesc &d = descs[g];
        const bool aligned = (reinterpret_cast<uintptr_t>(d.ptr) & 15u) == 0 && (d.ld & 3) == 0;
        if (aligned || d.n < 2) continue;
        which.push_back(g);
        const int64_t ldw = ((int64_t)d.n + 3) & ~(int64_t)3;
        apsp::BatchCopy c{};
        c.user = d.ptr;
        c.work = reinterpret_cast<uint32_t *>(words);  // offset for now
        c.ld_user = d.ld;
        c.ld_work = ldw;
        c.row0 = rows;
        c.n = d.n;
        copies.push_back(c);
        words += (int64_t)d.n * ldw;
        rows += d.n;
    }
    if (copies.empty()) return;
    void *buf = nullptr;
    const size_t bytes = (size_t)words * sizeof(uint32_t);
    const hipError_t e = p->stream_ordered ? hipMallocAsync(&buf, bytes, s) : hipMalloc(&buf, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // no room: those graphs run in place
        copies.clear();
        return;
    }
    p->work = static_cast<uint32_t *>(buf);
    for (size_t k = 0; k < copies.size(); ++k) {
        copies[k].work = p->work + reinterpret_cast<int64_t>(copies[k].work);
        descs[which[k]].ptr = copies[k].work;
        descs[which[k]].ld = copies[k].ld_work;
    }
    p->copies = (int32_t)copies.size();
    p->copy_rows = rows;
}

// Create a plan; `stream_ordered` selects hipMallocAsync on `s` (one-shot use)
// instead of hipMalloc.
int32_t plan_create(void *const *ptrs, const int32_t *ns, const int64_t *lds, int32_t count,
                    int32_t dtype, int32_t tile, const int32_t *table, hipStream_t s,
                    bool stream_ordered, apsp_batch_plan **out) {
    *out = nullptr;
    if (tile != 0 && tile != 64 && tile != 128) return APSP_ERR_INVALID_VALUE;
    if (table)
        for (int b = 0; b < apsp::kTuneBuckets; ++b)
            if (table[b] != 64 && table[b] != 128) return APSP_ERR_INVALID_VALUE;
    const int32_t st = check_batch(ptrs, ns, lds, count, dtype);
    if (st != APSP_OK) return st;
    apsp_batch_plan *p = new (std::nothrow) apsp_batch_plan();
    if (!p) return APSP_ERR_NO_MEMORY;
    p->dtype = dtype;
    p->stream_ordered = stream_ordered;
    p->device = -1;
    // host tables in per-thread buffers that keep their capacity between
    // calls (a one-shot solve builds a plan per call)
    thread_local std::vector<apsp::BatchDesc> descs;
    thread_local std::vector<apsp::BatchItem> items;
    thread_local std::vector<unsigned char> host;
    thread_local std::vector<apsp::BatchCopy> copies;
    descs.clear();
    items.clear();
    copies.clear();
    if (count > 0) apsp::plan_build(*p, ptrs, ns, lds, count, tile, table, descs, items);
    if (!descs.empty()) {  // an empty batch makes no HIP call at all
        if (hipGetDevice(&p->device) != hipSuccess) {
            delete p;
            return APSP_ERR_DEVICE;
        }
        plan_working_copies(p, descs, copies, s);
        const TableLayout t = table_layout(descs.size(), items.size(), copies.size(), dtype);
        pack_tables(descs, items, copies, t, host);
        void *buf = nullptr;
        const hipError_t e =
            stream_ordered ? hipMallocAsync(&buf, t.total, s) : hipMalloc(&buf, t.total);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            free_plan_buffers(p, s);
            delete p;
            return APSP_ERR_NO_MEMORY;
        }
        point_tables(p, buf, t);
        // Pageable source: the copy has consumed the host buffer when it returns.
        if (hipMemcpyAsync(buf, host.data(), t.total, hipMemcpyHostToDevice, s) != hipSuccess ||
            (!stream_ordered && hipStreamSynchronize(s) != hipSuccess)) {
            free_plan_buffers(p, s);
            delete p;
            return APSP_ERR_DEVICE;
        }
    }
    *out = p;
    return APSP_OK;
}

int32_t plan_run(const apsp_batch_plan *p, hipStream_t s) {
    if (p->copies) {
        const hipError_t e =
            apsp::launch_batch_copies(p->d_copies, p->copies, p->copy_rows, false, s);
        if (e != hipSuccess) {
            apsp::note_error("batched working copies", e);
            return APSP_ERR_DEVICE;
        }
    }
    if (p->d_wmax) {
        const hipError_t e = apsp::launch_batched_wmax(p->d_descs, p->d_items, p->scan, p->d_wmax,
                                                       p->graphs, s);
        if (e != hipSuccess) {
            apsp::note_error("batched weight scan", e);
            return APSP_ERR_DEVICE;
        }
    }
    for (const auto &L : p->launches) {
        const hipError_t e = apsp::launch_batched_items(p->d_descs, p->d_items, L.ranges, L.r,
                                                        L.close_only, p->dtype, p->d_wmax, s);
        if (e != hipSuccess) {
            apsp::note_error("batched launch", e);
            return APSP_ERR_DEVICE;
        }
    }
    if (p->copies) {
        const hipError_t e =
            apsp::launch_batch_copies(p->d_copies, p->copies, p->copy_rows, true, s);
        if (e != hipSuccess) {
            apsp::note_error("batched working copies (back)", e);
            return APSP_ERR_DEVICE;
        }
    }
    return APSP_OK;
}

}  // namespace

int32_t apsp::batched_plan_create_table(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                        int32_t count, int32_t dtype, const int32_t *table,
                                        hipStream_t s, apsp_batch_plan **out) {
    if (out == nullptr || table == nullptr) return APSP_ERR_INVALID_VALUE;
    return plan_create(ptrs, ns, lds, count, dtype, 0, table, s, false, out);
}

extern "C" {

int32_t apsp_batched_plan_create(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                 int32_t count, int32_t dtype, void *stream,
                                 apsp_batch_plan **plan) {
    if (plan == nullptr) return APSP_ERR_INVALID_VALUE;
    return plan_create(ptrs, ns, lds, count, dtype, 0, nullptr,
                       reinterpret_cast<hipStream_t>(stream), false, plan);
}

int32_t apsp_batched_plan_create_tiled(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                       int32_t count, int32_t dtype, int32_t tile, void *stream,
                                       apsp_batch_plan **plan) {
    if (plan == nullptr) return APSP_ERR_INVALID_VALUE;
    return plan_create(ptrs, ns, lds, count, dtype, tile, nullptr,
                       reinterpret_cast<hipStream_t>(stream), false, plan);
}

int32_t apsp_batched_plan_run(const apsp_batch_plan *plan, void *stream) {
    if (plan == nullptr) return APSP_ERR_INVALID_VALUE;
    return plan_run(plan, reinterpret_cast<hipStream_t>(stream));
}

int32_t apsp_batched_plan_info(const apsp_batch_plan *plan, int64_t *info) {
    if (plan == nullptr || info == nullptr) return APSP_ERR_INVALID_VALUE;
    info[0] = (int64_t)plan->launches.size();
    info[1] = plan->items;
    info[2] = plan->tiles;
    return APSP_OK;
}

int32_t apsp_batched_plan_destroy(apsp_batch_plan *plan) {
    if (plan == nullptr) return APSP_OK;
    if (plan->device >= 0) {
        int cur = 0;
        const bool have = hipGetDevice(&cur) == hipSuccess;
        if (have && cur != plan->device) (void)hipSetDevice(plan->device);
        free_plan_buffers(plan, nullptr);
        if (have && cur != plan->device) (void)hipSetDevice(cur);
    }
    delete plan;
    return APSP_OK;
}

int32_t apsp_solve_batched_ex(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                              int32_t count, int32_t dtype, void *stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    apsp_batch_plan *p = nullptr;
    const int32_t st = plan_create(ptrs, ns, lds, count, dtype, 0, nullptr, s, true, &p);
    if (st != APSP_OK) return st;
    const int32_t rs = plan_run(p, s);
    free_plan_buffers(p, s);  // stream-ordered: freed after the launches
    delete p;
    return rs;
}

int32_t apsp_solve_batched(void *const *ptrs, const int32_t *ns, int32_t count, void *stream) {
    return apsp_solve_batched_ex(ptrs, ns, nullptr, count, APSP_I32, stream);
}

}  // extern "C"

// ---- allocation-free batched solve ------------------------------------------
// apsp_solve_batched_noalloc keeps its tables in this file-scope device array
// instead of memory it allocates.  Each GPU the library runs on has its own
// copy, held until the process ends.  Host code never passes the array's name
// to a kernel or a copy (on the host it only names the symbol): it uses the
// device address hipGetSymbolAddress returns, looked up once per device.
namespace {

constexpr size_t kNoAllocBytes = (size_t)APSP_NOALLOC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxScratchDevices] = {};

// The current device's copy of `scratch` (its device address), or null.
void *scratch_for_current_device(hipError_t *err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= kMaxScratchDevices)) e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        *err = e;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            *err = e != hipSuccess ? e : hipErrorInvalidSymbol;
            return nullptr;
        }
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" int32_t apsp_solve_batched_noalloc(void *const *ptrs, const int32_t *ns,
                                              const int64_t *lds, int32_t count, int32_t dtype,
                                              void *stream) {
    const int32_t st = check_batch(ptrs, ns, lds, count, dtype);
    if (st != APSP_OK) return st;
    if (count == 0) return APSP_OK;
    // host tables in per-thread buffers that keep their capacity between calls
    thread_local std::vector<apsp::BatchDesc> descs;
    thread_local std::vector<apsp::BatchItem> items;
    thread_local std::vector<unsigned char> host;
    apsp_batch_plan p;
    p.dtype = dtype;
    apsp::plan_build(p, ptrs, ns, lds, count, 0, nullptr, descs, items);
    if (descs.empty()) return APSP_OK;  // every graph empty: no HIP call
    const TableLayout t = table_layout(descs.size(), items.size(), 0, dtype);
    if (t.total > kNoAllocBytes) {
        char msg[160];
        snprintf(msg, sizeof(msg),
                 "batch tables need %zu bytes; the allocation-free workspace holds %zu",
                 t.total, kNoAllocBytes);
        apsp::note_message(msg);
        return APSP_ERR_UNSUPPORTED;
    }
    hipError_t e = hipSuccess;
    void *ws = scratch_for_current_device(&e);
    if (!ws) {
        apsp::note_error("hipGetSymbolAddress(scratch)", e);
        return APSP_ERR_DEVICE;
    }
    thread_local std::vector<apsp::BatchCopy> no_copies;  // no working copies here
    pack_tables(descs, items, no_copies, t, host);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // Pageable source: the copy has consumed the host buffer when it returns.
    e = hipMemcpyAsync(ws, host.data(), t.total, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) {
        apsp::note_error("hipMemcpyAsync to the allocation-free workspace", e);
        return APSP_ERR_DEVICE;
    }
    point_tables(&p, ws, t);
    return plan_run(&p, s);
}

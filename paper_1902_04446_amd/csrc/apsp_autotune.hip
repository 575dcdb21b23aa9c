// Batched tuning table: the round width (64 or 128) that the batched path
// uses for a graph, per device and per size bucket, and two autotuners that
// fill it: one times both widths on synthetic batches of each bucket, the
// other a given batch (on copies) under greedy per-bucket choices.
//
// Buckets: b = 0..7 hold n in (64b, 64b + 64]; bucket 8 holds n > 512.
// Within a bucket both widths run the same number of rounds (ceil(n/64) and
// ceil(n/128) are constant over it), so one representative size per bucket
// (its upper end; 1024 for bucket 8) decides it.  Until a device is tuned
// (or its table set) every bucket uses 128.
#include <algorithm>
#include <atomic>
#include <vector>

#include "../../include/apsp.h"
#include "apsp_common.h"

namespace apsp {

namespace {

constexpr int kMaxDevices = 64;
std::atomic<int> g_table[kMaxDevices][kTuneBuckets];  // 0 = unset (128)

int64_t bucket_size(int b) { return b < 8 ? 64 * (int64_t)(b + 1) : 1024; }

bool current_device(int *dev) {
    if (hipGetDevice(dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return *dev >= 0 && *dev < kMaxDevices;
}

// Synthetic dense weights (timing only; the kernels are branch-free, so the
// values do not change the work): the murmur3 32-bit finaliser of the index,
// as int32 in [1, 1024] or fp32 in [1, 2).
__global__ void k_fill_synth(uint32_t *buf, int64_t count, uint32_t seed, int dtype) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        uint32_t h = (uint32_t)i * 0x9e3779b1u ^ (uint32_t)(i >> 32) ^ seed;
        h ^= h >> 16;
        h *= 0x85ebca6bu;
        h ^= h >> 13;
        h *= 0xc2b2ae35u;
        h ^= h >> 16;
        buf[i] = dtype == 0 ? (h & 0x3ffu) + 1u : ((h >> 9) | 0x3f800000u);
    }
}

}  // namespace

int batched_bucket(int64_t n) { return n <= 512 ? (n <= 64 ? 0 : (int)((n - 1) / 64)) : 8; }

void batched_tuning_snapshot(int32_t *table) {
    int dev = 0;
    const bool have = current_device(&dev);
    for (int b = 0; b < kTuneBuckets; ++b) {
        const int v = have ? g_table[dev][b].load(std::memory_order_relaxed) : 0;
        table[b] = v == 64 ? 64 : kRoundB;
    }
}

int batched_tile(int64_t n) {
    int dev = 0;
    if (!current_device(&dev)) return kRoundB;
    const int v = g_table[dev][batched_bucket(n < 1 ? 1 : n)].load(std::memory_order_relaxed);
    return v == 64 ? 64 : kRoundB;
}

}  // namespace apsp

namespace {

struct Scratch {
    void *buf = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    apsp_batch_plan *plan = nullptr;
    ~Scratch() {
        if (plan) apsp_batched_plan_destroy(plan);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (buf) (void)hipFree(buf);
    }
};

// Average milliseconds of one run of a `tile`-wide plan over `graphs` graphs
// of n vertices stored back to back in buf; < 0 on failure (status in *st).
double time_plan(Scratch &S, int64_t n, int64_t graphs, int32_t dtype, int32_t tile, int reps,
                 hipStream_t s, int32_t *st) {
    std::vector<void *> ptrs((size_t)graphs);
    std::vector<int32_t> ns((size_t)graphs, (int32_t)n);
    for (int64_t g = 0; g < graphs; ++g)
        ptrs[(size_t)g] = static_cast<uint32_t *>(S.buf) + g * n * n;
    *st = apsp_batched_plan_create_tiled(ptrs.data(), ns.data(), nullptr, (int32_t)graphs, dtype,
                                         tile, s, &S.plan);
    if (*st != APSP_OK) return -1.0;
    *st = apsp_batched_plan_run(S.plan, s);  // warm-up
    if (*st == APSP_OK && hipEventRecord(S.e0, s) != hipSuccess) *st = APSP_ERR_DEVICE;
    for (int i = 0; i < reps && *st == APSP_OK; ++i) *st = apsp_batched_plan_run(S.plan, s);
    if (*st == APSP_OK && hipEventRecord(S.e1, s) != hipSuccess) *st = APSP_ERR_DEVICE;
    if (*st == APSP_OK && hipEventSynchronize(S.e1) != hipSuccess) *st = APSP_ERR_DEVICE;
    float ms = 0.0f;
    if (*st == APSP_OK && hipEventElapsedTime(&ms, S.e0, S.e1) != hipSuccess) *st = APSP_ERR_DEVICE;
    apsp_batched_plan_destroy(S.plan);
    S.plan = nullptr;
    return *st == APSP_OK ? (double)ms / reps : -1.0;
}

}  // namespace

extern "C" {

int32_t apsp_batched_tuning_get(int32_t *table, int32_t count) {
    if (table == nullptr || count != APSP_TUNE_BUCKETS) return APSP_ERR_INVALID_VALUE;
    int dev = 0;
    if (!apsp::current_device(&dev)) return APSP_ERR_DEVICE;
    for (int b = 0; b < APSP_TUNE_BUCKETS; ++b) {
        const int v = apsp::g_table[dev][b].load(std::memory_order_relaxed);
        table[b] = v == 64 ? 64 : apsp::kRoundB;
    }
    return APSP_OK;
}

int32_t apsp_batched_tuning_set(const int32_t *table, int32_t count) {
    if (table == nullptr || count != APSP_TUNE_BUCKETS) return APSP_ERR_INVALID_VALUE;
    for (int b = 0; b < APSP_TUNE_BUCKETS; ++b)
        if (table[b] != 64 && table[b] != 128) return APSP_ERR_INVALID_VALUE;
    int dev = 0;
    if (!apsp::current_device(&dev)) return APSP_ERR_DEVICE;
    for (int b = 0; b < APSP_TUNE_BUCKETS; ++b)
        apsp::g_table[dev][b].store(table[b], std::memory_order_relaxed);
    return APSP_OK;
}

int32_t apsp_batched_autotune(int32_t dtype, int64_t batch_elems, void *stream, int32_t *table,
                              double *ms) {
    if (dtype != APSP_I32 && dtype != APSP_F32) return APSP_ERR_INVALID_VALUE;
    if (batch_elems < ((int64_t)1 << 20) || batch_elems > ((int64_t)1 << 30))
        return APSP_ERR_INVALID_VALUE;
    int dev = 0;
    if (!apsp::current_device(&dev)) return APSP_ERR_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Scratch S;
    if (hipMalloc(&S.buf, (size_t)batch_elems * 4) != hipSuccess) {
        (void)hipGetLastError();
        return APSP_ERR_NO_MEMORY;
    }
    if (hipEventCreate(&S.e0) != hipSuccess || hipEventCreate(&S.e1) != hipSuccess)
        return APSP_ERR_DEVICE;
    hipLaunchKernelGGL(apsp::k_fill_synth, dim3(4096), dim3(256), 0, s,
                       static_cast<uint32_t *>(S.buf), batch_elems, 0x1902u, (int)dtype);
    if (hipGetLastError() != hipSuccess) return APSP_ERR_DEVICE;
    int32_t result[APSP_TUNE_BUCKETS];
    for (int b = 0; b < APSP_TUNE_BUCKETS; ++b) {
        const int64_t n = apsp::bucket_size(b);
        const int64_t graphs = batch_elems / (n * n);
        if (graphs < 1) return APSP_ERR_INVALID_VALUE;
        int32_t st = APSP_OK;
        const double t128 = time_plan(S, n, graphs, dtype, 128, 3, s, &st);
        if (st != APSP_OK) return st;
        const double t64 = time_plan(S, n, graphs, dtype, 64, 3, s, &st);
        if (st != APSP_OK) return st;
        // 64 only on a clear win: the two are equal work on even bucket ends
        result[b] = t64 < 0.97 * t128 ? 64 : 128;
        if (ms) {
            ms[2 * b] = t128;
            ms[2 * b + 1] = t64;
        }
    }
    for (int b = 0; b < APSP_TUNE_BUCKETS; ++b) {
        apsp::g_table[dev][b].store(result[b], std::memory_order_relaxed);
        if (table) table[b] = result[b];
    }
    return APSP_OK;
}

int32_t apsp_batched_autotune_batch(void *const *ptrs, const int32_t *ns, const int64_t *lds,
                                    int32_t count, int32_t dtype, void *stream, int32_t *table,
                                    double *ms) {
    if (dtype != APSP_I32 && dtype != APSP_F32) return APSP_ERR_INVALID_VALUE;
    if (count <= 0 || ptrs == nullptr || ns == nullptr) return APSP_ERR_INVALID_VALUE;
    std::vector<int64_t> off((size_t)count + 1, 0), ldw((size_t)count);
    double work[APSP_TUNE_BUCKETS] = {0};
    for (int32_t g = 0; g < count; ++g) {
        const int64_t n = ns[g];
        const int64_t ld = lds ? lds[g] : (n > 1 ? n : 1);
        if (n < 0 || n > APSP_BATCHED_MAX_N || ld < (n > 1 ? n : 1)) return APSP_ERR_INVALID_VALUE;
        if (n > 0 && ptrs[g] == nullptr) return APSP_ERR_INVALID_VALUE;
        ldw[(size_t)g] = n > 0 ? (n + 3) / 4 * 4 : 1;  // 16-byte rows in the copies
        off[(size_t)g + 1] = off[(size_t)g] + n * ldw[(size_t)g];
        if (n > 0) work[apsp::batched_bucket(n)] += (double)n * n * n;
    }
    const int64_t total = off[(size_t)count];
    if (total == 0) return APSP_ERR_INVALID_VALUE;
    int dev = 0;
    if (!apsp::current_device(&dev)) return APSP_ERR_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Scratch S;   // S.buf: the working copy, then the pristine copy
    if (hipMalloc(&S.buf, (size_t)total * 8) != hipSuccess) {
        (void)hipGetLastError();
        return APSP_ERR_NO_MEMORY;
    }
    if (hipEventCreate(&S.e0) != hipSuccess || hipEventCreate(&S.e1) != hipSuccess)
        return APSP_ERR_DEVICE;
    uint32_t *wk = static_cast<uint32_t *>(S.buf), *pristine = wk + total;
    std::vector<void *> wptr((size_t)count);
    for (int32_t g = 0; g < count; ++g) {
        wptr[(size_t)g] = wk + off[(size_t)g];
        const int64_t n = ns[g];
        if (n == 0) continue;
        const int64_t ld = lds ? lds[g] : (n > 1 ? n : 1);
        if (hipMemcpy2DAsync(pristine + off[(size_t)g], (size_t)ldw[(size_t)g] * 4, ptrs[g],
                             (size_t)ld * 4, (size_t)n * 4, (size_t)n, hipMemcpyDeviceToDevice,
                             s) != hipSuccess)
            return APSP_ERR_DEVICE;
    }
    // milliseconds of one solve of the copies with the given widths (best of 5,
    // each from the pristine inputs)
    auto timed = [&](const int32_t *tab, double *out) -> int32_t {
        int32_t st = apsp::batched_plan_create_table(wptr.data(), ns, ldw.data(), count, dtype, tab,
                                                     s, &S.plan);
        double best = -1.0;
        for (int rep = 0; rep < 5 && st == APSP_OK; ++rep) {
            float t = 0.0f;
            if (hipMemcpyAsync(wk, pristine, (size_t)total * 4, hipMemcpyDeviceToDevice, s) !=
                    hipSuccess ||
                hipEventRecord(S.e0, s) != hipSuccess) {
                st = APSP_ERR_DEVICE;
                break;
            }
            st = apsp_batched_plan_run(S.plan, s);
            if (st == APSP_OK && (hipEventRecord(S.e1, s) != hipSuccess ||
                                  hipEventSynchronize(S.e1) != hipSuccess ||
                                  hipEventElapsedTime(&t, S.e0, S.e1) != hipSuccess))
                st = APSP_ERR_DEVICE;
            if (st == APSP_OK && (best < 0 || t < best)) best = t;
        }
        if (S.plan) apsp_batched_plan_destroy(S.plan);
        S.plan = nullptr;
        *out = best;
        return st;
    };
    int32_t cur[APSP_TUNE_BUCKETS];
    for (int b = 0; b < APSP_TUNE_BUCKETS; ++b) cur[b] = 128;
    double base = 0.0;
    int32_t st = timed(cur, &base);
    if (st != APSP_OK) return st;
    double best = base;
    // greedy: buckets in decreasing order of their share of the work
    int order[APSP_TUNE_BUCKETS];
    for (int b = 0; b < APSP_TUNE_BUCKETS; ++b) order[b] = b;
    std::sort(order, order + APSP_TUNE_BUCKETS, [&](int a, int b) { return work[a] > work[b]; });
    for (int i = 0; i < APSP_TUNE_BUCKETS; ++i) {
        const int b = order[i];
        if (work[b] == 0.0) continue;
        cur[b] = 64;
        double t = 0.0;
        st = timed(cur, &t);
        if (st != APSP_OK) return st;
        if (t < 0.97 * best)
            best = t;
        else
            cur[b] = 128;
    }
    for (int b = 0; b < APSP_TUNE_BUCKETS; ++b) {
        apsp::g_table[dev][b].store(cur[b], std::memory_order_relaxed);
        if (table) table[b] = cur[b];
    }
    if (ms) {
        ms[0] = base;
        ms[1] = best;
    }
    return APSP_OK;
}

}  // extern "C"

// VALU issue-rate probe (diagnostic library, not part of the solver).
//
// Measures the lane-instruction throughput of the instructions the min-plus
// kernels are built from, and of their mix as the tile update issues it, so
// the benchmark can state the ceilings it compares against on the machine it
// runs on.  Each thread runs 16 independent
// register-only dependency chains of one instruction (inline asm on registers
// only: no memory operand), for `iters` iterations, across a grid large
// enough to fill every SIMD.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <int MODE>
__global__ __launch_bounds__(256) void k_probe(uint32_t *out, int iters, uint32_t seed) {
    uint32_t a[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = seed + threadIdx.x * 16u + (uint32_t)i;
    const uint32_t b = seed * 3u + 1u, c = seed * 5u + 7u;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (MODE == 0) asm volatile("v_add_f32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
            if (MODE == 1) asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
            if (MODE == 2) asm volatile("v_min3_i32 %0, %0, %1, %2" : "+v"(a[i]) : "v"(b), "v"(c));
            if (MODE == 3) asm volatile("v_min3_u32 %0, %0, %1, %2" : "+v"(a[i]) : "v"(b), "v"(c));
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) s ^= a[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// The update mix itself: per 4 output cells, 8 fp32 adds then 4 v_min3_i32,
// c = min3(c, x + y, x' + y'), 16 cells per thread (2 updates per cell and
// iteration), registers only.
__global__ __launch_bounds__(256) void k_mix(uint32_t *out, int iters, uint32_t seed) {
    uint32_t c[16], x[4], x2[4], y[4], y2[4];
#pragma unroll
    for (int i = 0; i < 16; ++i) c[i] = 0x7f000000u + threadIdx.x + (uint32_t)i;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        x[i] = __float_as_uint(1.0f + (float)(i + seed));
        x2[i] = __float_as_uint(2.0f + (float)i);
        y[i] = __float_as_uint(0.5f + (float)(i * threadIdx.x));
        y2[i] = __float_as_uint(0.25f + (float)i);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            uint32_t t0, t1, t2, t3, t4, t5, t6, t7;
            asm volatile(
                "v_add_f32 %0, %12, %14\n v_add_f32 %1, %13, %18\n"
                "v_add_f32 %2, %12, %15\n v_add_f32 %3, %13, %19\n"
                "v_add_f32 %4, %12, %16\n v_add_f32 %5, %13, %20\n"
                "v_add_f32 %6, %12, %17\n v_add_f32 %7, %13, %21\n"
                "v_min3_i32 %8, %8, %0, %1\n v_min3_i32 %9, %9, %2, %3\n"
                "v_min3_i32 %10, %10, %4, %5\n v_min3_i32 %11, %11, %6, %7\n"
                : "=&v"(t0), "=&v"(t1), "=&v"(t2), "=&v"(t3), "=&v"(t4), "=&v"(t5), "=&v"(t6),
                  "=&v"(t7), "+v"(c[m * 4 + 0]), "+v"(c[m * 4 + 1]), "+v"(c[m * 4 + 2]),
                  "+v"(c[m * 4 + 3])
                : "v"(x[m]), "v"(x2[m]), "v"(y[0]), "v"(y[1]), "v"(y[2]), "v"(y[3]), "v"(y2[0]),
                  "v"(y2[1]), "v"(y2[2]), "v"(y2[3]));
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) s ^= c[i];
    out[blockIdx.x * 256 + threadIdx.x] = s;
}

// Cell updates per second of the update mix (after a warm-up long enough
// for the clock to settle).
double mix_rate(uint32_t *out, int grid, int iters) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    hipLaunchKernelGGL(k_mix, dim3(grid), dim3(256), 0, 0, out, iters, 1u);
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL(k_mix, dim3(grid), dim3(256), 0, 0, out, iters, 1u);
    (void)hipEventRecord(e1, 0);
    float ms = 0.f;
    double r = -1.0;
    if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
        ms > 0.f)
        r = (double)grid * 256.0 * iters * 32.0 / (ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
}

template <int MODE>
double rate(uint32_t *out, int grid, int iters) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.0;
    hipLaunchKernelGGL(k_probe<MODE>, dim3(grid), dim3(256), 0, 0, out, 8, 1u);
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL(k_probe<MODE>, dim3(grid), dim3(256), 0, 0, out, iters, 1u);
    (void)hipEventRecord(e1, 0);
    float ms = 0.f;
    double r = -1.0;
    if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
        ms > 0.f)
        r = (double)grid * 256.0 * iters * 16.0 / (ms * 1e-3);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return r;
}

}  // namespace

extern "C" {

// Writes lane-instructions per second for v_add_f32, v_add_u32, v_min3_i32,
// v_min3_u32 into rates[0..3] (on the current device, default stream;
// synchronous).  Returns 0 on success, -1 on a HIP failure.
int apsp_probe_valu_rates(double *rates);

// Cell updates per second of the register-only update mix (2 fp32 adds +
// 1 v_min3_i32 per 2 updates) into *rate.  Returns 0 on success.
int apsp_probe_update_mix(double *rate) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    const int grid = cus * 32;
    uint32_t *out = nullptr;
    if (hipMalloc(&out, sizeof(uint32_t) * (size_t)grid * 256) != hipSuccess) return -1;
    *rate = mix_rate(out, grid, 4000);
    (void)hipFree(out);
    return *rate > 0 ? 0 : -1;
}

int apsp_probe_valu_rates(double *rates) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return -1;
    const int grid = cus * 32;  // 32 workgroups of 4 waves per CU: every SIMD saturated
    uint32_t *out = nullptr;
    if (hipMalloc(&out, sizeof(uint32_t) * (size_t)grid * 256) != hipSuccess) return -1;
    const int iters = 20000;
    rates[0] = rate<0>(out, grid, iters);
    rates[1] = rate<1>(out, grid, iters);
    rates[2] = rate<2>(out, grid, iters);
    rates[3] = rate<3>(out, grid, iters);
    (void)hipFree(out);
    for (int i = 0; i < 4; ++i)
        if (rates[i] <= 0) return -1;
    return 0;
}
}

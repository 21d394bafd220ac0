// Machine ceilings measured on the device the library runs on, for the
// roofline fractions the benchmark reports: HBM bandwidth (STREAM-style copy
// and triad over arrays far larger than the caches), FP64 vector FMA rate
// and FP64 matrix-core rate (v_mfma_f64_16x16x4f64 back to back from
// registers).  Diagnostic only; nothing on the solver path uses it.
#include "pqph_internal.h"

#include <vector>

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_stream_copy(const double2* __restrict__ a, double2* __restrict__ b,
                                                     long n2) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x)
        b[i] = a[i];
}

__global__ __launch_bounds__(256) void k_stream_triad(double2* __restrict__ a, const double2* __restrict__ b,
                                                      const double2* __restrict__ c, double s, long n2) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
        const double2 x = b[i], y = c[i];
        a[i] = double2{x.x + s * y.x, x.y + s * y.y};
    }
}

// 8 independent FMA chains per thread, ITER steps each: 16 * ITER flop per thread
constexpr int FMA_ITER = 4096;
__global__ __launch_bounds__(256) void k_fma_peak(double* __restrict__ out, double seed) {
    double v[8];
    for (int j = 0; j < 8; ++j) v[j] = seed + threadIdx.x * 1e-9 + j;
    const double m = 1.0 - 1e-12, c = 1e-13;
    for (int it = 0; it < FMA_ITER; ++it)
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = __builtin_fma(v[j], m, c);
    double s = 0.0;
    for (int j = 0; j < 8; ++j) s += v[j];
    if (s == 12345.678) out[0] = s;      // keeps the chains live; never true in practice
}

// 4 independent accumulators per wavefront, ITER MFMA steps each; one
// 16x16x4 FP64 MFMA is 2 * 16 * 16 * 4 = 2048 flop
constexpr int MFMA_ITER = 2048;
__global__ __launch_bounds__(256) void k_mfma_peak(double* __restrict__ out, double seed) {
    const double a = seed + threadIdx.x * 1e-9, b = 1.0 - 1e-12;
    d4 acc[4];
    for (int u = 0; u < 4; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < MFMA_ITER; ++it)
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
    double s = 0.0;
    for (int u = 0; u < 4; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
    if (s == 12345.678) out[0] = s;
}

}  // namespace

extern "C" pqph_status pqph_measure_ceilings(pqph_ctx* ctx, double* out) {
    if (!ctx) return pqph_fail(nullptr, PQPH_INVALID_ARG, "null context");
    if (!out) return pqph_fail(ctx, PQPH_INVALID_ARG, "null output");
    PQPH_HIP(ctx, hipSetDevice(ctx->device));
    const long n = 1L << 27;       // 1 GiB per array: far beyond L2 and MALL
    const size_t bytes = (size_t)n * sizeof(double);
    pqph_status st = pqph_ensure_ws(ctx, 3 * bytes);
    if (st) return st;
    double* a = ctx->ws;
    double* b = a + n;
    double* c = b + n;
    hipStream_t s = ctx->stream;
    PQPH_HIP(ctx, hipMemsetAsync(a, 0, 3 * bytes, s));
    const long n2 = n / 2;
    const int grid = 256 * 16;
    auto timed = [&](auto launch, int reps, float& ms) -> pqph_status {
        launch();                                   // warm-up
        PQPH_HIP(ctx, hipEventRecord(ctx->ev0, s));
        for (int r = 0; r < reps; ++r) launch();
        PQPH_HIP(ctx, hipEventRecord(ctx->ev1, s));
        PQPH_HIP(ctx, hipEventSynchronize(ctx->ev1));
        PQPH_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ms /= reps;
        return PQPH_OK;
    };
    float ms = 0.f;
    if ((st = timed([&] { hipLaunchKernelGGL(k_stream_copy, dim3(grid), dim3(256), 0, s,
                                             (const double2*)a, (double2*)b, n2); }, 10, ms)))
        return st;
    out[0] = 2.0 * bytes / (ms * 1e-3) / 1e9;
    if ((st = timed([&] { hipLaunchKernelGGL(k_stream_triad, dim3(grid), dim3(256), 0, s, (double2*)a,
                                             (const double2*)b, (const double2*)c, 0.5, n2); }, 10, ms)))
        return st;
    out[1] = 3.0 * bytes / (ms * 1e-3) / 1e9;
    const int blocks = 256 * 8;                     // 8 workgroups of 4 waves per CU
    if ((st = timed([&] { hipLaunchKernelGGL(k_fma_peak, dim3(blocks), dim3(256), 0, s, a, 1.0); }, 5, ms)))
        return st;
    out[2] = (double)blocks * 256 * 16.0 * FMA_ITER / (ms * 1e-3) / 1e12;
    if ((st = timed([&] { hipLaunchKernelGGL(k_mfma_peak, dim3(blocks), dim3(256), 0, s, a, 1.0); }, 5, ms)))
        return st;
    out[3] = (double)blocks * 4 * 4 * 2048.0 * MFMA_ITER / (ms * 1e-3) / 1e12;
    PQPH_HIP(ctx, hipGetLastError());
    return PQPH_OK;
}

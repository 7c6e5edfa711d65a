// Measured ceilings of the device, for the rooflines the benchmark reports
// beside the datasheet figures: the FP64 and FP32 matrix-core rates
// (independent v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32 chains in
// every wave, two waves per SIMD) and the HBM rate of a plain copy (each
// byte read once and written once, 16-byte accesses, grid-stride).  The copy
// is also the reference for scaling the hardware byte counters.
#include <string>
#include <vector>
#include <algorithm>
#include "internal.h"

namespace {

constexpr int PK_CHAINS = 8;  // independent accumulators per wave

template <class T>
__global__ __launch_bounds__(256) void mfma_peak_kernel(int iters, T seed, T* out) {
    typedef typename std::conditional<sizeof(T) == 8, d4_t, f4_t>::type acc_t;
    acc_t acc[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) acc[c] = acc_t{0, 0, 0, 0};
    T a = seed * (T)(threadIdx.x & 15), b = seed * (T)(threadIdx.x >> 4);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < PK_CHAINS; ++c) {
            if constexpr (sizeof(T) == 8)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
            else
                acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
        }
    }
    T s = 0;
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void copy_peak_kernel(int64_t n2, const double2* __restrict__ a,
                                                        double2* __restrict__ b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

template <class F>
int time_ms(fl_ctx* ctx, int reps, F launch, double* best_ms) {
    hipEvent_t e0, e1;
    FL_HIP(ctx, hipEventCreate(&e0));
    FL_HIP(ctx, hipEventCreate(&e1));
    std::vector<float> t;
    hipError_t err = hipSuccess;
    for (int r = 0; r <= reps && err == hipSuccess; ++r) {
        err = hipEventRecord(e0, ctx->stream);
        if (err == hipSuccess) err = launch();
        if (err == hipSuccess) err = hipEventRecord(e1, ctx->stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float ms = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (r > 0) t.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fl_fail(ctx, FL_EHIP, std::string("peak measurement: ") + hipGetErrorString(err));
    *best_ms = *std::min_element(t.begin(), t.end());
    return FL_OK;
}

}  // namespace

extern "C" {

int fl_measure_peaks(fl_ctx* ctx, double* fp64_tflops, double* fp32_tflops, double* copy_gbs, int64_t copy_bytes) {
    if (!ctx) return FL_EINVAL;
    if (copy_gbs && copy_bytes < (1 << 20)) return fl_fail(ctx, FL_EINVAL, "fl_measure_peaks: copy of at least 1 MiB");
    FL_HIP(ctx, hipSetDevice(ctx->device));
    hipDeviceProp_t prop;
    FL_HIP(ctx, hipGetDeviceProperties(&prop, ctx->device));
    const int blocks = prop.multiProcessorCount * 2;  // 256 threads = 4 waves: two per SIMD with 2 blocks/CU
    const int iters = 4096;
    DevBuf out;
    FL_HIP(ctx, out.alloc((size_t)blocks * 256 * 8));
    const double flops = 2.0 * 16 * 16 * 4 * PK_CHAINS * (double)iters * (blocks * 4);
    double ms = 0;
    int rc;
    if (fp64_tflops) {
        rc = time_ms(ctx, 5, [&]() {
            mfma_peak_kernel<double><<<blocks, 256, 0, ctx->stream>>>(iters, 1e-3, out.as<double>());
            return hipGetLastError();
        }, &ms);
        if (rc) return rc;
        *fp64_tflops = flops / (ms * 1e-3) / 1e12;
    }
    if (fp32_tflops) {
        rc = time_ms(ctx, 5, [&]() {
            mfma_peak_kernel<float><<<blocks, 256, 0, ctx->stream>>>(iters, 1e-3f, out.as<float>());
            return hipGetLastError();
        }, &ms);
        if (rc) return rc;
        *fp32_tflops = flops / (ms * 1e-3) / 1e12;
    }
    if (copy_gbs) {
        const int64_t n2 = copy_bytes / 16;
        DevBuf a, b;
        FL_HIP(ctx, a.alloc((size_t)n2 * 16));
        FL_HIP(ctx, b.alloc((size_t)n2 * 16));
        FL_HIP(ctx, hipMemsetAsync(a.p, 0, (size_t)n2 * 16, ctx->stream));
        const int cblocks = prop.multiProcessorCount * 16;
        rc = time_ms(ctx, 5, [&]() {
            copy_peak_kernel<<<cblocks, 256, 0, ctx->stream>>>(n2, a.as<double2>(), b.as<double2>());
            return hipGetLastError();
        }, &ms);
        if (rc) return rc;
        *copy_gbs = 2.0 * (double)n2 * 16 / (ms * 1e-3) / 1e9;
    }
    return FL_OK;
}

}  // extern "C"

// Measured ceilings of the device, for the rooflines the benchmark reports
// beside the datasheet figures: the FP64 and FP32 matrix-core rates
// (independent v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32 chains in
// every wave; 8 or 16 chains, 2 or 4 waves per SIMD, the best of the four)
// and the HBM rate of a plain copy (each byte read once and written once,
// four 16-byte accesses in flight per thread, grid-stride; the best of
// 8 and 32 workgroups per CU).  The copy is also the reference for scaling
// the hardware byte counters.
#include <string>
#include <vector>
#include <algorithm>
#include "internal.h"

namespace {

template <class T, int PK_CHAINS>
__global__ __launch_bounds__(256) void mfma_peak_kernel(int iters, T seed, T* out) {
    typedef typename std::conditional<sizeof(T) == 8, d4_t, f4_t>::type acc_t;
    acc_t acc[PK_CHAINS];
#pragma unroll
    for (int c = 0; c < PK_CHAINS; ++c) acc[c] = acc_t{0, 0, 0, 0};
    T a = seed * (T)(threadIdx.x & 15), b = seed * (T)(threadIdx.x >> 4);
    // eight rounds per trip (iters is a multiple of 8), so that moving the
    // loop-carried accumulators between register files is amortised
    for (int i = 0; i < iters; i += 8) {
#pragma unroll
        for (int r = 0; r < 8; ++r)
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

// n2 a multiple of 4 * 256 * gridDim.x is not required: the tail loop
// copies what the unrolled part leaves.
__global__ __launch_bounds__(256) void copy_peak_kernel(int64_t n2, const double2* __restrict__ a,
                                                        double2* __restrict__ b) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * stride < n2; i += 4 * stride) {
        const double2 x0 = a[i], x1 = a[i + stride], x2 = a[i + 2 * stride], x3 = a[i + 3 * stride];
        b[i] = x0;
        b[i + stride] = x1;
        b[i + 2 * stride] = x2;
        b[i + 3 * stride] = x3;
    }
    for (; i < n2; i += stride) b[i] = a[i];
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
    const int iters = 2048;
    DevBuf out;
    FL_HIP(ctx, out.alloc((size_t)prop.multiProcessorCount * 4 * 256 * 8));
    double ms = 0;
    int rc;
    // best over (chains, waves per SIMD); 256 threads = 4 waves per workgroup
    auto best_rate = [&](auto launch_for, double* result) -> int {
        double best = 0.0;
        for (int wps : {2, 4}) {
            const int blocks = prop.multiProcessorCount * wps;
            for (int chains : {8, 16}) {
                int r = time_ms(ctx, 5, [&]() { return launch_for(blocks, chains); }, &ms);
                if (r) return r;
                const double flops = 2.0 * 16 * 16 * 4 * chains * (double)iters * (blocks * 4);
                best = std::max(best, flops / (ms * 1e-3) / 1e12);
            }
        }
        *result = best;
        return FL_OK;
    };
    if (fp64_tflops) {
        rc = best_rate([&](int blocks, int chains) {
            if (chains == 8)
                mfma_peak_kernel<double, 8><<<blocks, 256, 0, ctx->stream>>>(iters, 1e-3, out.as<double>());
            else
                mfma_peak_kernel<double, 16><<<blocks, 256, 0, ctx->stream>>>(iters, 1e-3, out.as<double>());
            return hipGetLastError();
        }, fp64_tflops);
        if (rc) return rc;
    }
    if (fp32_tflops) {
        rc = best_rate([&](int blocks, int chains) {
            if (chains == 8)
                mfma_peak_kernel<float, 8><<<blocks, 256, 0, ctx->stream>>>(iters, 1e-3f, out.as<float>());
            else
                mfma_peak_kernel<float, 16><<<blocks, 256, 0, ctx->stream>>>(iters, 1e-3f, out.as<float>());
            return hipGetLastError();
        }, fp32_tflops);
        if (rc) return rc;
    }
    if (copy_gbs) {
        const int64_t n2 = copy_bytes / 16;
        DevBuf a, b;
        FL_HIP(ctx, a.alloc((size_t)n2 * 16));
        FL_HIP(ctx, b.alloc((size_t)n2 * 16));
        FL_HIP(ctx, hipMemsetAsync(a.p, 0, (size_t)n2 * 16, ctx->stream));
        double best = 0.0;
        for (int per_cu : {8, 32}) {
            const int cblocks = prop.multiProcessorCount * per_cu;
            rc = time_ms(ctx, 5, [&]() {
                copy_peak_kernel<<<cblocks, 256, 0, ctx->stream>>>(n2, a.as<double2>(), b.as<double2>());
                return hipGetLastError();
            }, &ms);
            if (rc) return rc;
            best = std::max(best, 2.0 * (double)n2 * 16 / (ms * 1e-3) / 1e9);
        }
        *copy_gbs = best;
    }
    return FL_OK;
}

}  // extern "C"

// Spectral application that allocates nothing, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// Its intermediates G = M F, C = V^T G, the weights W and the split-k
// partial sums of V^T G live in one file-scope device array of fixed size
// (FL_NOALLOC_SCRATCH_BYTES), which each device holds until the process
// ends.  Host code never passes the array's name to a kernel: its device
// address is taken once per device with hipGetSymbolAddress (at the first
// call on that device, with the device current) and only that address is
// used.  Every call on a device shares the device's array, so calls that
// overlap on one device (on different streams, or from different threads)
// race; calls on one stream are ordered.  Each call overwrites the whole
// part of the array it uses before reading it, so nothing needs clearing.
#include <mutex>
#include <string>
#include "internal.h"

static constexpr size_t SCRATCH_DOUBLES = FL_NOALLOC_SCRATCH_BYTES / sizeof(double);
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace {

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
double* g_scratch[MAX_DEVICES] = {nullptr};

// Device address of the scratch array on ctx's device, resolved once per
// device with that device current.
int scratch_address(fl_ctx* ctx, double** out) {
    *out = nullptr;
    if (ctx->device < 0 || ctx->device >= MAX_DEVICES)
        return fl_fail(ctx, FL_EINVAL, "scratch address: device ordinal out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[ctx->device]) {
        FL_HIP(ctx, hipSetDevice(ctx->device));
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fl_fail(ctx, FL_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[ctx->device] = static_cast<double*>(p);
    }
    *out = g_scratch[ctx->device];
    return FL_OK;
}

}  // namespace

extern "C" {

int fl_apply_fractional_noalloc(fl_op* op, int64_t nf, const double* F, int64_t ldf, int64_t na, const double* alpha,
                                int paired, double* U, int64_t ldu) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    const int64_t n = op->n;
    if (!op->has_eig) return fl_fail(ctx, FL_ESTATE, "fl_apply_fractional_noalloc: eigensolve first");
    if (nf <= 0 || na <= 0 || !F || !U || !alpha || ldf < n || ldu < n)
        return fl_fail(ctx, FL_EINVAL, "fl_apply_fractional_noalloc: bad sizes or null pointer");
    if (paired && nf != na) return fl_fail(ctx, FL_EINVAL, "fl_apply_fractional_noalloc: paired requires nf == na");
    for (int64_t i = 0; i < na; ++i)
        if (!(alpha[i] >= 0.0 && alpha[i] <= 2.0))
            return fl_fail(ctx, FL_EINVAL, "fl_apply_fractional_noalloc: alpha must lie in [0, 2]");
    const size_t need = fl_spectral_ws_doubles(n, nf, na);
    if (need > SCRATCH_DOUBLES)
        return fl_fail(ctx, FL_EINVAL,
                       "fl_apply_fractional_noalloc: needs " + std::to_string(need * 8) + " bytes of scratch ((2 nf + na) n " +
                           "doubles); the limit is " + std::to_string(FL_NOALLOC_SCRATCH_BYTES) + " bytes");
    double* base = nullptr;
    int rc = scratch_address(ctx, &base);
    if (rc) return rc;
    FL_HIP(ctx, hipSetDevice(ctx->device));
    // what the intermediates leave free takes the split-k partial sums of V^T G
    SplitWs split{base + need, (SCRATCH_DOUBLES - need) * sizeof(double)};
    SpecCall c{FL_SPEC_FRACTIONAL, nf, F, ldf, na, alpha, nullptr, paired, U, ldu};
    FL_HIP(ctx, fl_queue_spectral(op, ctx->stream, c, base, &split, false));
    return FL_OK;
}

}  // extern "C"

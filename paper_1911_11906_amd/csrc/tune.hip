// Launch-shape autotuner for the matrix-core products.
//
// A table maps a product shape to the launch shape measured fastest for it:
// plain FP64/FP32 products (128 x 128 tiles with k-step 16 or 32, or
// 256 x 64 tiles for products with at most 64 columns, each optionally split
// along k) and the fused spectral-application product (k-step 16 or 32,
// XCD-grouped tile order with 4, 8 or 16 row tiles per band).  Shapes match
// on (kind, ta, tb, m, n) and on k's power-of-two bucket.  fl_gemm_tune times
// every candidate on the context's stream (HIP events, median of `reps` after
// one warm-up) and records the fastest; the table can be read out and set
// again so that a caller can keep it between processes.  Every launcher
// consults the table first and falls back to its built-in heuristics.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>
#include "internal.h"

namespace {

struct Entry {
    fl_gemm_choice c;
    int kbucket;
};

std::mutex g_mu;
std::vector<Entry> g_table;
std::atomic<int64_t> g_count{0};

int kbucket(int64_t k) {
    int b = 0;
    while ((int64_t(1) << b) < k && b < 62) ++b;
    return b;
}

bool valid_choice(const fl_gemm_choice& c) {
    if (c.kind != FL_TUNE_F64 && c.kind != FL_TUNE_F32 && c.kind != FL_TUNE_SCALED) return false;
    if (c.variant < FL_GV_AUTO || c.variant > FL_GV_THIN) return false;
    if (c.kind == FL_TUNE_SCALED && c.variant == FL_GV_THIN) return false;
    if (c.split < 1 || c.split > 64 || c.group < 1 || c.group > 64) return false;
    return c.m > 0 && c.n > 0 && c.k > 0;
}

void record(const fl_gemm_choice& c) {
    std::lock_guard<std::mutex> lk(g_mu);
    const int kb = kbucket(c.k);
    for (Entry& e : g_table)
        if (e.c.kind == c.kind && e.c.ta == c.ta && e.c.tb == c.tb && e.c.m == c.m && e.c.n == c.n && e.kbucket == kb) {
            e.c = c;
            return;
        }
    g_table.push_back(Entry{c, kb});
    g_count.store((int64_t)g_table.size());
}

__global__ void pattern_kernel(int64_t count, uint64_t seed, double* out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i < count; i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t z = (uint64_t)i * 0x9E3779B97F4A7C15ull + seed;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        out[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
    }
}

hipError_t fill_pattern(hipStream_t s, size_t count, uint64_t seed, double* out) {
    pattern_kernel<<<1024, 256, 0, s>>>((int64_t)count, seed, out);
    return hipGetLastError();
}

}  // namespace

GemmChoice tuned_choice(int kind, int ta, int tb, int64_t m, int64_t n, int64_t k) {
    GemmChoice r;
    if (g_count.load(std::memory_order_relaxed) == 0) return r;
    const int kb = kbucket(k);
    std::lock_guard<std::mutex> lk(g_mu);
    for (const Entry& e : g_table)
        if (e.c.kind == kind && e.c.ta == ta && e.c.tb == tb && e.c.m == m && e.c.n == n && e.kbucket == kb) {
            r.variant = e.c.variant;
            r.split = e.c.split;
            r.group = e.c.group;
            break;
        }
    return r;
}

extern "C" {

int fl_gemm_tune(fl_ctx* ctx, int kind, int ta, int tb, int64_t m, int64_t n, int64_t k, int reps,
                 fl_gemm_choice* best) {
    if (!ctx) return FL_EINVAL;
    if (!best || m <= 0 || n <= 0 || k <= 0 || reps < 1 || reps > 100 ||
        (kind != FL_TUNE_F64 && kind != FL_TUNE_F32 && kind != FL_TUNE_SCALED))
        return fl_fail(ctx, FL_EINVAL, "fl_gemm_tune: bad arguments");
    if (kind == FL_TUNE_SCALED && k != m) return fl_fail(ctx, FL_EINVAL, "fl_gemm_tune: the spectral product has k == m");
    FL_HIP(ctx, hipSetDevice(ctx->device));
    hipStream_t s = ctx->stream;
    // candidates
    std::vector<GemmChoice> cand;
    if (kind == FL_TUNE_SCALED) {
        for (int v : {FL_GV_SQUARE16, FL_GV_SQUARE32})
            for (int g : {4, 8, 16}) {
                GemmChoice c;
                c.variant = v;
                c.group = g;
                cand.push_back(c);
            }
    } else {
        const int maxs = (int)std::min<int64_t>(32, std::max<int64_t>(1, k / 128));
        if (n <= 64)
            for (int sp = 1; sp <= maxs; sp *= 2) {
                GemmChoice c;
                c.variant = FL_GV_THIN;
                c.split = sp;
                cand.push_back(c);
            }
        for (int sp = 1; sp <= std::min(maxs, 8); sp *= 2) {
            GemmChoice c;
            c.variant = FL_GV_SQUARE16;
            c.split = sp;
            cand.push_back(c);
        }
        GemmChoice c;
        c.variant = FL_GV_SQUARE32;
        cand.push_back(c);
    }
    // operands
    const size_t esz = kind == FL_TUNE_F32 ? 4 : 8;
    int64_t nf = n, na = 1;
    if (kind == FL_TUNE_SCALED && n % 1024 == 0) {
        nf = 1024;
        na = n / 1024;
    }
    const size_t a_elems = (size_t)m * k;
    const size_t b_elems = kind == FL_TUNE_SCALED ? (size_t)k * (nf + na) : (size_t)k * n;
    const size_t c_elems = (size_t)m * n;
    DevBuf bA, bB, bC;
    FL_HIP(ctx, bA.alloc(a_elems * esz));
    FL_HIP(ctx, bB.alloc(b_elems * esz));
    FL_HIP(ctx, bC.alloc(c_elems * esz));
    // FP32 operands are filled through their bytes as doubles (values do not matter)
    FL_HIP(ctx, fill_pattern(s, a_elems * esz / 8, 1, bA.as<double>()));
    FL_HIP(ctx, fill_pattern(s, b_elems * esz / 8, 2, bB.as<double>()));
    if (kind == FL_TUNE_SCALED) {
        // weights in (0, 1]
        FL_HIP(ctx, fl_fill(s, k, na, 0.5, bB.as<double>() + (size_t)k * nf, k));
    }
    hipEvent_t e0, e1;
    FL_HIP(ctx, hipEventCreate(&e0));
    FL_HIP(ctx, hipEventCreate(&e1));
    double best_ms = 1e300;
    GemmChoice bestc;
    hipError_t err = hipSuccess;
    for (const GemmChoice& c : cand) {
        std::vector<float> t;
        for (int r = 0; r <= reps && err == hipSuccess; ++r) {
            err = hipEventRecord(e0, s);
            if (err != hipSuccess) break;
            if (kind == FL_TUNE_SCALED) {
                const double* V = bA.as<double>();
                const double* C = bB.as<double>();
                const double* W = C + (size_t)k * nf;
                err = fl_scaled_gemm(s, m, V, m, W, k, C, k, nf, na, 0, bC.as<double>(), m, &c, false);
            } else {
                const int64_t lda = ta ? k : m, ldb = tb ? n : k;
                err = fl_gemm_choice_launch(s, kind, ta, tb, m, n, k, bA.p, lda, bB.p, ldb, bC.p, m, c);
            }
            if (err == hipSuccess) err = hipEventRecord(e1, s);
            if (err == hipSuccess) err = hipEventSynchronize(e1);
            float ms = 0.f;
            if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            if (r > 0) t.push_back(ms);
        }
        if (err != hipSuccess) break;
        std::sort(t.begin(), t.end());
        const double med = t[t.size() / 2];
        if (med < best_ms) {
            best_ms = med;
            bestc = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fl_fail(ctx, FL_EHIP, std::string("fl_gemm_tune: ") + hipGetErrorString(err));
    fl_gemm_choice out{};
    out.kind = kind;
    out.ta = kind == FL_TUNE_SCALED ? 0 : ta;
    out.tb = kind == FL_TUNE_SCALED ? 0 : tb;
    out.m = m;
    out.n = n;
    out.k = k;
    out.variant = bestc.variant;
    out.split = bestc.split;
    out.group = bestc.group;
    out.ms = best_ms;
    record(out);
    *best = out;
    return FL_OK;
}

int fl_gemm_tuning_set(const fl_gemm_choice* c) {
    if (!c || !valid_choice(*c)) return FL_EINVAL;
    record(*c);
    return FL_OK;
}

int64_t fl_gemm_tuning_count(void) { return g_count.load(); }

int fl_gemm_tuning_get(int64_t i, fl_gemm_choice* out) {
    if (!out) return FL_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || i >= (int64_t)g_table.size()) return FL_EINVAL;
    *out = g_table[i].c;
    return FL_OK;
}

void fl_gemm_tuning_clear(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_table.clear();
    g_count.store(0);
}

}  // extern "C"

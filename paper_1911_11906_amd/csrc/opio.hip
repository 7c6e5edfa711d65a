// Saving and loading an operator with its eigenbasis, so that the basis is
// computed once and reused for every later forcing (Section "Method", the
// paragraph after the equation for v: the expensive part is finding the
// eigenpairs, after which each solve is a sum over them).
//
// File layout (little-endian, as the host writes it):
//   "FRACLAP\0", u32 version (1), u32 flags (bit 0: eigenpairs present;
//   bit 1: the operator keeps no dense pencil),
//   i64 n, i64 nnz, i32 precision (FL_FP64, FL_MIXED or -1), i32 refinement
//   steps, f64 last refinement residual, 32-byte SHA-256 of the pencil
//   (the CSR arrays below, in order), then the CSR arrays
//   rowptr (n + 1 i32), colidx (nnz i32), K values (nnz f64), M values
//   (nnz f64), then theta (n f64) and V (n x n f64, column-major, ld = n)
//   when present, and a 32-byte SHA-256 of every preceding byte.
// The dense K and M of a loaded operator (unless bit 1 is set) are scattered
// back from the CSR arrays on the device (they hold exactly the pattern's
// entries).
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include "internal.h"

namespace {

// SHA-256 (FIPS 180-4).
struct Sha256 {
    uint32_t h[8];
    uint8_t buf[64];
    uint64_t len = 0;
    size_t fill = 0;
    static constexpr uint32_t K[64] = {
        0x428a2f98, 0x71374491, 0xb5c0fbcf, 0xe9b5dba5, 0x3956c25b, 0x59f111f1, 0x923f82a4, 0xab1c5ed5,
        0xd807aa98, 0x12835b01, 0x243185be, 0x550c7dc3, 0x72be5d74, 0x80deb1fe, 0x9bdc06a7, 0xc19bf174,
        0xe49b69c1, 0xefbe4786, 0x0fc19dc6, 0x240ca1cc, 0x2de92c6f, 0x4a7484aa, 0x5cb0a9dc, 0x76f988da,
        0x983e5152, 0xa831c66d, 0xb00327c8, 0xbf597fc7, 0xc6e00bf3, 0xd5a79147, 0x06ca6351, 0x14292967,
        0x27b70a85, 0x2e1b2138, 0x4d2c6dfc, 0x53380d13, 0x650a7354, 0x766a0abb, 0x81c2c92e, 0x92722c85,
        0xa2bfe8a1, 0xa81a664b, 0xc24b8b70, 0xc76c51a3, 0xd192e819, 0xd6990624, 0xf40e3585, 0x106aa070,
        0x19a4c116, 0x1e376c08, 0x2748774c, 0x34b0bcb5, 0x391c0cb3, 0x4ed8aa4a, 0x5b9cca4f, 0x682e6ff3,
        0x748f82ee, 0x78a5636f, 0x84c87814, 0x8cc70208, 0x90befffa, 0xa4506ceb, 0xbef9a3f7, 0xc67178f2};
    Sha256() {
        const uint32_t h0[8] = {0x6a09e667, 0xbb67ae85, 0x3c6ef372, 0xa54ff53a,
                                0x510e527f, 0x9b05688c, 0x1f83d9ab, 0x5be0cd19};
        std::memcpy(h, h0, sizeof(h));
    }
    static uint32_t rotr(uint32_t x, int r) { return (x >> r) | (x << (32 - r)); }
    void block(const uint8_t* p) {
        uint32_t w[64];
        for (int i = 0; i < 16; ++i)
            w[i] = (uint32_t)p[4 * i] << 24 | (uint32_t)p[4 * i + 1] << 16 | (uint32_t)p[4 * i + 2] << 8 | p[4 * i + 3];
        for (int i = 16; i < 64; ++i) {
            uint32_t s0 = rotr(w[i - 15], 7) ^ rotr(w[i - 15], 18) ^ (w[i - 15] >> 3);
            uint32_t s1 = rotr(w[i - 2], 17) ^ rotr(w[i - 2], 19) ^ (w[i - 2] >> 10);
            w[i] = w[i - 16] + s0 + w[i - 7] + s1;
        }
        uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
        for (int i = 0; i < 64; ++i) {
            uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
            uint32_t ch = (e & f) ^ (~e & g);
            uint32_t t1 = hh + S1 + ch + K[i] + w[i];
            uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
            uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
            uint32_t t2 = S0 + mj;
            hh = g;
            g = f;
            f = e;
            e = d + t1;
            d = c;
            c = b;
            b = a;
            a = t1 + t2;
        }
        h[0] += a; h[1] += b; h[2] += c; h[3] += d;
        h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
    }
    void update(const void* data, size_t n) {
        const uint8_t* p = static_cast<const uint8_t*>(data);
        len += n;
        if (fill) {
            size_t take = std::min(n, 64 - fill);
            std::memcpy(buf + fill, p, take);
            fill += take;
            p += take;
            n -= take;
            if (fill == 64) {
                block(buf);
                fill = 0;
            }
        }
        while (n >= 64) {
            block(p);
            p += 64;
            n -= 64;
        }
        if (n) {
            std::memcpy(buf, p, n);
            fill = n;
        }
    }
    void final(uint8_t out[32]) {
        const uint64_t bits = len * 8;
        const uint8_t one = 0x80, zero = 0;
        update(&one, 1);
        while (fill != 56) update(&zero, 1);
        uint8_t lb[8];
        for (int i = 0; i < 8; ++i) lb[i] = (uint8_t)(bits >> (56 - 8 * i));
        update(lb, 8);
        for (int i = 0; i < 8; ++i)
            for (int j = 0; j < 4; ++j) out[4 * i + j] = (uint8_t)(h[i] >> (24 - 8 * j));
    }
};
constexpr uint32_t Sha256::K[64];

constexpr char MAGIC[8] = {'F', 'R', 'A', 'C', 'L', 'A', 'P', 0};
constexpr uint32_t VERSION = 1;

struct Header {
    char magic[8];
    uint32_t version;
    uint32_t flags;
    int64_t n;
    int64_t nnz;
    int32_t precision;
    int32_t refine_iters;
    double refine_resid;
    uint8_t pencil_sha[32];
};
static_assert(sizeof(Header) == 80, "file header layout");

// Writes through the running checksum.
struct Writer {
    FILE* f;
    Sha256 sha;
    bool ok = true;
    void put(const void* p, size_t n) {
        if (!ok || n == 0) return;
        sha.update(p, n);
        ok = std::fwrite(p, 1, n, f) == n;
    }
};
struct Reader {
    FILE* f;
    Sha256 sha;
    bool ok = true;
    void get(void* p, size_t n) {
        if (!ok || n == 0) return;
        ok = std::fread(p, 1, n, f) == n;
        if (ok) sha.update(p, n);
    }
};

__global__ void csr_scatter_kernel(int64_t n, const int32_t* __restrict__ rowptr, const int32_t* __restrict__ colidx,
                                   const double* __restrict__ kval, const double* __restrict__ mval, int64_t ld,
                                   double* __restrict__ K, double* __restrict__ M) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int32_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
        const int64_t j = colidx[p];
        K[i + j * ld] = kval[p];
        M[i + j * ld] = mval[p];
    }
}

template <class T>
int dalloc(fl_ctx* ctx, T** p, size_t count) {
    *p = nullptr;
    if (hipMalloc((void**)p, sizeof(T) * (count > 0 ? count : 1)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fl_fail(ctx, FL_ENOMEM, "device allocation of " + std::to_string(sizeof(T) * count) + " bytes failed");
    }
    return FL_OK;
}

}  // namespace

extern "C" {

int fl_op_save(const fl_op* op, const char* path) {
    if (!op) return FL_EINVAL;
    fl_ctx* ctx = op->ctx;
    if (!path || !op->rowptr) return fl_fail(ctx, FL_EINVAL, "fl_op_save: null path or operator without a pattern");
    FL_HIP(ctx, hipSetDevice(op->device));
    const int64_t n = op->n, nnz = op->nnz;
    std::vector<int32_t> rowptr(n + 1), colidx(nnz);
    std::vector<double> kval(nnz), mval(nnz), theta, V;
    hipStream_t s = ctx->stream;
    FL_HIP(ctx, hipMemcpyAsync(rowptr.data(), op->rowptr, 4 * (n + 1), hipMemcpyDeviceToHost, s));
    FL_HIP(ctx, hipMemcpyAsync(colidx.data(), op->colidx, 4 * nnz, hipMemcpyDeviceToHost, s));
    FL_HIP(ctx, hipMemcpyAsync(kval.data(), op->kval, 8 * nnz, hipMemcpyDeviceToHost, s));
    FL_HIP(ctx, hipMemcpyAsync(mval.data(), op->mval, 8 * nnz, hipMemcpyDeviceToHost, s));
    if (op->has_eig) {
        theta.resize(n);
        V.resize((size_t)n * n);
        FL_HIP(ctx, hipMemcpyAsync(theta.data(), op->theta, 8 * n, hipMemcpyDeviceToHost, s));
        FL_HIP(ctx, hipMemcpy2DAsync(V.data(), n * 8, op->V, op->ld * 8, n * 8, n, hipMemcpyDeviceToHost, s));
    }
    FL_HIP(ctx, hipStreamSynchronize(s));
    Header h{};
    std::memcpy(h.magic, MAGIC, 8);
    h.version = VERSION;
    h.flags = (op->has_eig ? 1u : 0u) | (op->K ? 0u : 2u);
    h.n = n;
    h.nnz = nnz;
    h.precision = op->eig_precision;
    h.refine_iters = op->refine_iters;
    h.refine_resid = op->refine_resid;
    {
        Sha256 ps;
        ps.update(rowptr.data(), 4 * (n + 1));
        ps.update(colidx.data(), 4 * nnz);
        ps.update(kval.data(), 8 * nnz);
        ps.update(mval.data(), 8 * nnz);
        ps.final(h.pencil_sha);
    }
    const std::string tmp = std::string(path) + ".part";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return fl_fail(ctx, FL_EIO, std::string("fl_op_save: cannot open ") + tmp);
    Writer w{f};
    w.put(&h, sizeof(h));
    w.put(rowptr.data(), 4 * (n + 1));
    w.put(colidx.data(), 4 * nnz);
    w.put(kval.data(), 8 * nnz);
    w.put(mval.data(), 8 * nnz);
    if (op->has_eig) {
        w.put(theta.data(), 8 * n);
        w.put(V.data(), 8 * V.size());
    }
    uint8_t dig[32];
    w.sha.final(dig);
    if (w.ok) w.ok = std::fwrite(dig, 1, 32, f) == 32;
    if (std::fclose(f) != 0) w.ok = false;
    if (!w.ok || std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fl_fail(ctx, FL_EIO, std::string("fl_op_save: writing ") + path + " failed");
    }
    return FL_OK;
}

int fl_op_load(fl_ctx* ctx, const char* path, fl_op** out) {
    if (!ctx) return FL_EINVAL;
    if (!path || !out) return fl_fail(ctx, FL_EINVAL, "fl_op_load: null argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fl_fail(ctx, FL_EIO, std::string("fl_op_load: cannot open ") + path);
    Reader r{f};
    Header h{};
    r.get(&h, sizeof(h));
    auto bad = [&](const std::string& why) {
        std::fclose(f);
        return fl_fail(ctx, FL_EIO, std::string("fl_op_load: ") + path + ": " + why);
    };
    if (!r.ok || std::memcmp(h.magic, MAGIC, 8) != 0) return bad("not an operator file");
    if (h.version != VERSION) return bad("unsupported version " + std::to_string(h.version));
    if (h.n <= 0 || h.n > (int64_t(1) << 31) || h.nnz <= 0 || h.nnz > h.n * h.n || (h.flags & ~3u))
        return bad("corrupt header");
    const int64_t n = h.n, nnz = h.nnz;
    std::vector<int32_t> rowptr(n + 1), colidx(nnz);
    std::vector<double> kval(nnz), mval(nnz), theta, V;
    r.get(rowptr.data(), 4 * (n + 1));
    r.get(colidx.data(), 4 * nnz);
    r.get(kval.data(), 8 * nnz);
    r.get(mval.data(), 8 * nnz);
    if (h.flags & 1u) {
        theta.resize(n);
        V.resize((size_t)n * n);
        r.get(theta.data(), 8 * n);
        r.get(V.data(), 8 * V.size());
    }
    uint8_t dig[32], want[32];
    if (r.ok) r.sha.final(dig);
    const bool tail = r.ok && std::fread(want, 1, 32, f) == 32;
    std::fclose(f);
    if (!r.ok || !tail) return fl_fail(ctx, FL_EIO, std::string("fl_op_load: ") + path + ": truncated");
    if (std::memcmp(dig, want, 32) != 0) return fl_fail(ctx, FL_EIO, std::string("fl_op_load: ") + path + ": checksum mismatch");
    // structural checks of the pattern (the kernels index with it)
    if (rowptr[0] != 0 || rowptr[n] != nnz) return fl_fail(ctx, FL_EIO, "fl_op_load: corrupt row pointers");
    for (int64_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) return fl_fail(ctx, FL_EIO, "fl_op_load: corrupt row pointers");
    for (int64_t p = 0; p < nnz; ++p)
        if (colidx[p] < 0 || colidx[p] >= n) return fl_fail(ctx, FL_EIO, "fl_op_load: column index out of range");
    FL_HIP(ctx, hipSetDevice(ctx->device));
    fl_op* op = new fl_op();
    op->ctx = ctx;
    op->device = ctx->device;
    op->n = n;
    op->ld = ((n + 15) / 16) * 16;
    op->nnz = nnz;
    op->eig_precision = h.precision;
    op->refine_iters = h.refine_iters;
    op->refine_resid = h.refine_resid;
    const size_t nn = (size_t)op->ld * n;
    const bool dense = !(h.flags & 2u);
    int rc;
    if ((dense && ((rc = dalloc(ctx, &op->K, nn)) || (rc = dalloc(ctx, &op->M, nn)))) ||
        (rc = dalloc(ctx, &op->rowptr, n + 1)) ||
        (rc = dalloc(ctx, &op->colidx, nnz)) || (rc = dalloc(ctx, &op->kval, nnz)) ||
        (rc = dalloc(ctx, &op->mval, nnz)) ||
        ((h.flags & 1u) && ((rc = dalloc(ctx, &op->theta, n)) || (rc = dalloc(ctx, &op->logtheta, n)) ||
                            (rc = dalloc(ctx, &op->V, nn))))) {
        fl_op_destroy(op);
        return rc;
    }
    hipStream_t s = ctx->stream;
    hipError_t e = hipSuccess;
    if ((dense && ((e = hipMemsetAsync(op->K, 0, nn * 8, s)) || (e = hipMemsetAsync(op->M, 0, nn * 8, s)))) ||
        (e = hipMemcpyAsync(op->rowptr, rowptr.data(), 4 * (n + 1), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(op->colidx, colidx.data(), 4 * nnz, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(op->kval, kval.data(), 8 * nnz, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(op->mval, mval.data(), 8 * nnz, hipMemcpyHostToDevice, s))) {
        fl_op_destroy(op);
        return fl_fail(ctx, FL_EHIP, std::string("fl_op_load: ") + hipGetErrorString(e));
    }
    if (dense) {
        csr_scatter_kernel<<<(unsigned)FL_DIV_UP(n, 256), 256, 0, s>>>(n, op->rowptr, op->colidx, op->kval, op->mval,
                                                                         op->ld, op->K, op->M);
        e = hipGetLastError();
    }
    if (e == hipSuccess && (h.flags & 1u)) {
        if ((e = hipMemcpyAsync(op->theta, theta.data(), 8 * n, hipMemcpyHostToDevice, s)) == hipSuccess &&
            (e = hipMemcpy2DAsync(op->V, op->ld * 8, V.data(), n * 8, n * 8, n, hipMemcpyHostToDevice, s)) ==
                hipSuccess)
            e = fl_log_kernel(s, n, op->theta, op->logtheta);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        fl_op_destroy(op);
        return fl_fail(ctx, FL_EHIP, std::string("fl_op_load: ") + hipGetErrorString(e));
    }
    op->has_eig = (h.flags & 1u) ? 1 : 0;
    *out = op;
    return FL_OK;
}

int fl_op_info(const fl_op* op, int64_t* n, int* has_eig, int* precision, int* refine_iters, double* refine_resid) {
    if (!op) return FL_EINVAL;
    if (n) *n = op->n;
    if (has_eig) *has_eig = op->has_eig;
    if (precision) *precision = op->eig_precision;
    if (refine_iters) *refine_iters = op->refine_iters;
    if (refine_resid) *refine_resid = op->refine_resid;
    return FL_OK;
}

}  // extern "C"

// csr_io.hip -- the system (A, b, x) written to a binary CSR file (layout in include/pct.h).
//
// The device arrays go to disk through two pinned host buffers: while one buffer is
// written with fwrite, the next chunk is copied into the other on the caller's stream.
#include "../../include/pct.h"

#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

namespace {

constexpr size_t CHUNK = size_t(64) << 20;   // bytes per pinned buffer

inline int64_t align64(int64_t v) { return (v + 63) & ~int64_t(63); }

struct Writer {
    FILE *f = nullptr;
    hipStream_t s = nullptr;
    char *buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    int64_t pos = 0;   // bytes written so far

    pct_status open(const char *path, hipStream_t stream) {
        s = stream;
        f = fopen(path, "wb");
        if (!f) return PCT_EIO;
        for (int i = 0; i < 2; ++i) {
            if (hipHostMalloc((void **)&buf[i], CHUNK, hipHostMallocDefault) != hipSuccess) return PCT_EHIP;
            if (hipEventCreateWithFlags(&ev[i], hipEventDisableTiming) != hipSuccess) return PCT_EHIP;
        }
        return PCT_OK;
    }
    pct_status close_all() {
        pct_status st = PCT_OK;
        for (int i = 0; i < 2; ++i) {
            if (ev[i] && hipEventDestroy(ev[i]) != hipSuccess) st = PCT_EHIP;
            if (buf[i] && hipHostFree(buf[i]) != hipSuccess) st = PCT_EHIP;
        }
        if (f && fclose(f) != 0 && st == PCT_OK) st = PCT_EIO;
        return st;
    }
    pct_status host(const void *p, size_t n) {
        if (n && fwrite(p, 1, n, f) != n) return PCT_EIO;
        pos += (int64_t)n;
        return PCT_OK;
    }
    pct_status pad_to(int64_t off) {
        static const char zeros[64] = {0};
        while (pos < off) {
            const size_t k = (size_t)(off - pos) < sizeof zeros ? (size_t)(off - pos) : sizeof zeros;
            const pct_status st = host(zeros, k);
            if (st != PCT_OK) return st;
        }
        return PCT_OK;
    }
    // n bytes of device memory at p, double-buffered
    pct_status device(const void *p, size_t n) {
        const char *src = (const char *)p;
        const size_t nchunks = (n + CHUNK - 1) / CHUNK;
        if (nchunks == 0) return PCT_OK;
        auto issue = [&](size_t c) -> pct_status {
            const size_t off = c * CHUNK, len = (n - off) < CHUNK ? (n - off) : CHUNK;
            if (hipMemcpyAsync(buf[c & 1], src + off, len, hipMemcpyDeviceToHost, s) != hipSuccess) return PCT_EHIP;
            if (hipEventRecord(ev[c & 1], s) != hipSuccess) return PCT_EHIP;
            return PCT_OK;
        };
        pct_status st = issue(0);
        for (size_t c = 0; c < nchunks && st == PCT_OK; ++c) {
            if (c + 1 < nchunks) st = issue(c + 1);   // the other buffer was written out last step
            if (st != PCT_OK) break;
            if (hipEventSynchronize(ev[c & 1]) != hipSuccess) return PCT_EHIP;
            const size_t len = (n - c * CHUNK) < CHUNK ? (n - c * CHUNK) : CHUNK;
            st = host(buf[c & 1], len);
        }
        if (st != PCT_OK) (void)hipStreamSynchronize(s);   // no copy may still target a buffer
        return st;
    }
};

}  // namespace

extern "C" pct_status pct_csr_write(const char *path, const pct_csr *A, const float *x_dev, void *stream) {
    if (!path || !A || A->n_rows < 0 || A->n_cols < 1 || A->nnz < 0 || !A->row_ptr_dev) return PCT_EINVAL;
    if (A->val_dtype != PCT_F32 && A->val_dtype != PCT_F16) return PCT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = A->n_rows, n = A->n_cols;
    // nnz from the last row pointer (waits for the caller's work on the stream)
    int64_t nnz = 0;
    if (hipMemcpyAsync(&nnz, A->row_ptr_dev + m, sizeof nnz, hipMemcpyDeviceToHost, s) != hipSuccess) return PCT_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PCT_EHIP;
    if (nnz < 0 || nnz > A->nnz) return PCT_EINVAL;
    if (nnz > 0 && (!A->cols_dev || !A->vals_dev)) return PCT_EINVAL;
    const int64_t vb = A->val_dtype == PCT_F16 ? 2 : 4;
    int64_t off = 128;
    const int64_t o_rp = off;
    off = align64(off + 8 * (m + 1));
    const int64_t o_c = off;
    off = align64(off + 4 * nnz);
    const int64_t o_v = off;
    off = align64(off + vb * nnz);
    const int64_t o_b = A->b_dev ? off : 0;
    if (A->b_dev) off = align64(off + 4 * m);
    const int64_t o_x = x_dev ? off : 0;

    char hdr[128];
    memset(hdr, 0, sizeof hdr);
    memcpy(hdr, PCT_CSR_MAGIC, 8);
    const int64_t h64[3] = {m, n, nnz};
    memcpy(hdr + 8, h64, sizeof h64);
    const int32_t h32[2] = {A->val_dtype, 1};
    memcpy(hdr + 32, h32, sizeof h32);
    const int64_t offs[5] = {o_rp, o_c, o_v, o_b, o_x};
    memcpy(hdr + 40, offs, sizeof offs);

    Writer w;
    pct_status st = w.open(path, s);
    if (st == PCT_OK) st = w.host(hdr, sizeof hdr);
    if (st == PCT_OK) st = w.pad_to(o_rp);
    if (st == PCT_OK) st = w.device(A->row_ptr_dev, (size_t)(8 * (m + 1)));
    if (st == PCT_OK) st = w.pad_to(o_c);
    if (st == PCT_OK) st = w.device(A->cols_dev, (size_t)(4 * nnz));
    if (st == PCT_OK) st = w.pad_to(o_v);
    if (st == PCT_OK) st = w.device(A->vals_dev, (size_t)(vb * nnz));
    if (st == PCT_OK && A->b_dev) {
        st = w.pad_to(o_b);
        if (st == PCT_OK) st = w.device(A->b_dev, (size_t)(4 * m));
    }
    if (st == PCT_OK && x_dev) {
        st = w.pad_to(o_x);
        if (st == PCT_OK) st = w.device(x_dev, (size_t)(4 * n));
    }
    const pct_status cs = w.close_all();
    return st != PCT_OK ? st : cs;
}

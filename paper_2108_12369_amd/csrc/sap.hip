// sap.hip -- string-averaging projections (SAP, Sec. II-D) on a CSR system A x = b
// (see include/pct.h for the method and the arithmetic).
//
//   pct_sap_prepare : k_sap_prepare   one wavefront per row: checks its bounds and
//                                     columns, coefficient lambda / ||a_i||^2 (FP64 sum)
//   pct_sap_iterate : k_sap_string    one wavefront per string: y = x_k, then the
//                                     relaxed projection of every row of the string in
//                                     order; y in LDS (when n floats fit) or in the
//                                     workspace; y_t written to the workspace
//                     k_sap_average   x_{k+1}[j] = sum_t w_t y_t[j] in FP64, t in order
//
// A string is a chain of dependent row updates, so the parallelism is the number of
// strings; one wavefront walks a row's entries 64 at a time.  The rows' metadata is
// loaded 64 rows at a time (one row per lane) and the first entries of the next rows
// are always in flight (eight rows of 256 entries with the LDS iterate, four of 512 with
// the workspace iterate), so that the wave waits on the latency of HBM only once per
// several rows.
#include "../../include/pct.h"
#include "pct_device.h"
#include "pct_wave.h"

#include <hip/hip_fp16.h>
#include <math.h>
#include <string.h>

namespace pct {
namespace {

constexpr int SAP_WAVES_PREP = 4;   // waves per block of k_sap_prepare
// Ring of rows in flight: D rows ahead, the first PF chunks of 64 entries of each.  The
// LDS iterate takes short rows from a long ring; the workspace iterate (large grids, long
// curved rows) takes longer rows from a shorter ring.
template <bool LDS> struct Ring { static constexpr int D = 8, PF = 4; };
template <> struct Ring<false> { static constexpr int D = 4, PF = 8; };

struct SapLayout {
    size_t coef_off, w_off, y_off, total;
};

inline size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

SapLayout sap_layout(int64_t m, int32_t n, int32_t M) {
    SapLayout L;
    L.coef_off = 256;   // [0, 256): status word (same header as the simulator workspace)
    L.w_off = a256(L.coef_off + (size_t)m * sizeof(float));
    L.y_off = a256(L.w_off + (size_t)M * sizeof(double));
    L.total = L.y_off + (size_t)M * (size_t)n * sizeof(float);
    return L;
}

struct SapArgs {
    int64_t m, nnz;
    int32_t n, M;
    const int64_t *row_ptr;
    const int32_t *cols;
    const void *vals;
    const float *b;
    const int64_t *order;
    float *coef;
    int32_t *status;
};

template <typename VT> __device__ __forceinline__ float val_at(const void *v, int64_t e);
template <> __device__ __forceinline__ float val_at<float>(const void *v, int64_t e) {
    return ((const float *)v)[e];
}
template <> __device__ __forceinline__ float val_at<__half>(const void *v, int64_t e) {
    return __half2float(((const __half *)v)[e]);
}

// Row bounds clamped into [0, nnz]: a row whose stored bounds are outside is empty here
// (and was flagged by the prepare pass).
__device__ __forceinline__ void row_bounds(const SapArgs &a, int64_t i, int64_t &beg, int64_t &end) {
    beg = a.row_ptr[i];
    end = a.row_ptr[i + 1];
    if (beg < 0 || end < beg || end > a.nnz) {
        beg = 0;
        end = 0;
    }
}

template <typename VT>
__global__ __launch_bounds__(64 * SAP_WAVES_PREP) void k_sap_prepare(SapArgs a, float relax) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = (int64_t)blockIdx.x * SAP_WAVES_PREP + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * SAP_WAVES_PREP;
    for (int64_t i = wid; i < a.m; i += nw) {
        const int64_t beg = a.row_ptr[i], end = a.row_ptr[i + 1];
        bool ok = beg >= 0 && end >= beg && end <= a.nnz;
        double nrm = 0.0;
        if (ok) {
            for (int64_t e = beg + lane; e < end; e += 64) {
                const int32_t c = a.cols[e];
                ok = ok && (uint32_t)c < (uint32_t)a.n;
                const double v = (double)val_at<VT>(a.vals, e);
                nrm = fma(v, v, nrm);
            }
        }
        const bool all_ok = __builtin_amdgcn_ballot_w64(!ok) == 0;
        nrm = wave_sum(nrm);
        if (lane == 0) {
            a.coef[i] = (all_ok && nrm > 0.0) ? (float)((double)relax / nrm) : 0.0f;
            if (!all_ok) set_status_dev(a.status, PCT_EINVAL);
        }
        if (a.order && lane == 0) {
            const int64_t o = a.order[i];
            if (o < 0 || o >= a.m) set_status_dev(a.status, PCT_EINVAL);
        }
    }
}

// Metadata of one row of a string, fetched ahead.
struct RowMeta {
    int64_t beg, end;
    float b, coef;
};

__device__ __forceinline__ RowMeta fetch_meta(const SapArgs &a, int64_t s, int64_t s1) {
    RowMeta r{0, 0, 0.0f, 0.0f};
    if (s < s1) {
        const int64_t i = a.order ? a.order[s] : s;
        if (i >= 0 && i < a.m) {
            row_bounds(a, i, r.beg, r.end);
            r.b = a.b[i];
            r.coef = a.coef[i];
        }
    }
    return r;
}

// y[c] as the string sees it: LDS, or the workspace copy read at agent scope (past the
// non-coherent L1, so that the atomic adds of the previous row are seen).
template <bool LDS>
__device__ __forceinline__ float y_load(float *y, int32_t c) {
    if (LDS) return y[c];
    return __hip_atomic_load(y + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <bool LDS>
__device__ __forceinline__ void y_add(float *y, int32_t c, float v) {
    if (LDS) atomicAdd(y + c, v);   // ds_add_f32: entries of one row may share a voxel
    else unsafeAtomicAdd(y + c, v);
}

// Workspace iterate: the wave's adds (performed in L2) are complete before its next loads
// (which read L2).  The fence keeps the compiler from moving memory accesses across.
__device__ __forceinline__ void y_settle() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// First PF chunks of a row's entries.  The loads are unconditional (an index past the
// row reads a valid entry of the arrays, nnz > 0) so that nothing waits for them here;
// whether an entry belongs to the row is decided where it is used.
template <typename VT, int PF>
__device__ __forceinline__ void fetch_chunks(const SapArgs &a, const RowMeta &r, int lane, int32_t (&c)[PF],
                                             float (&v)[PF]) {
    const int64_t last = a.nnz - 1;
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int64_t e = r.beg + k * 64 + lane;
        const int64_t ec = e < last ? e : last;
        c[k] = a.cols[ec];
        v[k] = val_at<VT>(a.vals, ec);
    }
}

template <typename VT, bool LDS, int PF>
__device__ __forceinline__ void project_row(const SapArgs &a, float *y, const RowMeta &r, const int32_t (&cc)[PF],
                                            const float (&cv)[PF], int lane) {
    if (r.coef == 0.0f) return;
    const uint32_t n = (uint32_t)a.n;
    bool ok[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) ok[k] = r.beg + k * 64 + lane < r.end && (uint32_t)cc[k] < n;
    // all gathers of the prefetched chunks in flight before the first use; an entry past
    // the row or with a bad column reads y[0] and counts 0
    float yv[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) yv[k] = y_load<LDS>(y, ok[k] ? cc[k] : 0);
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < PF; ++k) acc = fma(ok[k] ? (double)cv[k] : 0.0, (double)yv[k], acc);
    for (int64_t e = r.beg + PF * 64 + lane; e < r.end; e += 64) {
        const int32_t c = a.cols[e];
        const bool okc = (uint32_t)c < n;
        const float yc = y_load<LDS>(y, okc ? c : 0);
        acc = fma(okc ? (double)val_at<VT>(a.vals, e) : 0.0, (double)yc, acc);
    }
    const double dot = wave_sum(acc);
    const float alpha = (float)(((double)r.b - dot) * (double)r.coef);
#pragma unroll
    for (int k = 0; k < PF; ++k)
        if (ok[k]) y_add<LDS>(y, cc[k], alpha * cv[k]);
    for (int64_t e = r.beg + PF * 64 + lane; e < r.end; e += 64) {
        const int32_t c = a.cols[e];
        if ((uint32_t)c < n) y_add<LDS>(y, c, alpha * val_at<VT>(a.vals, e));
    }
    // the next row's gathers must see these adds
    if (!LDS) y_settle();
}

// Metadata of 64 consecutive string positions, one per lane.
struct LaneMeta {
    int64_t beg, end;
    float b, coef;
};

__device__ __forceinline__ LaneMeta lane_meta(const SapArgs &a, int64_t base, int64_t s1, int lane) {
    const RowMeta r = fetch_meta(a, base + lane, s1);
    return LaneMeta{r.beg, r.end, r.b, r.coef};
}

// Position `idx` (uniform, < 64) of the lane-held metadata, as scalars.
__device__ __forceinline__ RowMeta meta_at(const LaneMeta &m, int idx) {
    RowMeta r;
    const uint64_t bg = (uint64_t)m.beg, en = (uint64_t)m.end;
    r.beg = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(bg >> 32), idx) << 32) |
                      (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)bg, idx));
    r.end = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(en >> 32), idx) << 32) |
                      (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)en, idx));
    r.b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, m.b), idx));
    r.coef = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, m.coef), idx));
    return r;
}

template <typename VT, bool LDS>
__global__ __launch_bounds__(64) void k_sap_string(SapArgs a, const float *x, float *Y) {
    extern __shared__ float ys[];
    constexpr int D = Ring<LDS>::D, PF = Ring<LDS>::PF;
    const int lane = threadIdx.x;
    const int t = blockIdx.x;
    const int n = a.n;
    float *yg = Y + (size_t)t * (size_t)n;
    float *y = LDS ? ys : yg;
    for (int j = lane; j < n; j += 64) y[j] = x[j];
    if (!LDS) y_settle();
    __syncthreads();

    // The string's positions go in batches of 64 whose metadata the lanes hold (this
    // batch in A, the next one in B).  Slot j of the ring holds the first PF chunks of
    // the row at position j (mod D); a slot is refilled with the row D positions on as
    // soon as its row is projected, so the loads of D rows are always in flight.
    const int64_t s0 = (int64_t)t * a.m / a.M, s1 = (int64_t)(t + 1) * a.m / a.M;
    LaneMeta A = lane_meta(a, s0, s1, lane), B = lane_meta(a, s0 + 64, s1, lane);
    int32_t cq[D][PF];
    float vq[D][PF];
#pragma unroll
    for (int j = 0; j < D; ++j) fetch_chunks<VT, PF>(a, meta_at(A, j), lane, cq[j], vq[j]);
    for (int64_t sb = s0; sb < s1; sb += 64) {
        for (int j0 = 0; j0 < 64; j0 += D) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                project_row<VT, LDS, PF>(a, y, meta_at(A, j0 + j), cq[j], vq[j], lane);
                const int nx = j0 + j + D;   // the position D on, in this batch or the next
                const RowMeta mn = nx < 64 ? meta_at(A, nx) : meta_at(B, nx - 64);
                fetch_chunks<VT, PF>(a, mn, lane, cq[j], vq[j]);
            }
        }
        A = B;
        B = lane_meta(a, sb + 128, s1, lane);
    }
    if (LDS) {
        __syncthreads();
        for (int j = lane; j < n; j += 64) yg[j] = ys[j];
    }
}

__global__ void k_sap_average(const float *Y, const double *w, int32_t M, int32_t n, float *x) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int32_t t = 0; t < M; ++t) s = fma(w[t], (double)Y[(size_t)t * (size_t)n + (size_t)j], s);
    x[j] = (float)s;
}

__global__ void k_sap_uniform(double *w, int32_t M) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < M) w[t] = 1.0 / (double)M;
}

__global__ void k_sap_clear_status(int32_t *status) {
    if (threadIdx.x == 0) *status = PCT_OK;
}

pct_status check_sap(const pct_csr *A, const pct_sap *p) {
    if (!A || !p) return PCT_EINVAL;
    if (A->n_rows < 0 || A->n_cols < 1 || A->nnz < 0) return PCT_EINVAL;
    if (A->val_dtype != PCT_F32 && A->val_dtype != PCT_F16) return PCT_EINVAL;
    if (!A->row_ptr_dev) return PCT_EINVAL;
    if (A->n_rows > 0 && (!A->b_dev || (A->nnz > 0 && (!A->cols_dev || !A->vals_dev)))) return PCT_EINVAL;
    if (p->n_strings < 1) return PCT_EINVAL;
    if (!(p->relax > 0.0f && p->relax < 2.0f)) return PCT_EINVAL;
    if (p->weights) {
        double sum = 0.0;
        for (int32_t t = 0; t < p->n_strings; ++t) {
            const double w = p->weights[t];
            if (!(w >= 0.0) || !isfinite(w)) return PCT_EINVAL;
            sum += w;
        }
        if (!(fabs(sum - 1.0) <= 1e-9)) return PCT_EINVAL;
    }
    // (t + 1) * m must not overflow int64; the string iterates must be addressable
    if ((double)A->n_rows * (double)p->n_strings > 9.0e18) return PCT_ERANGE;
    if ((double)p->n_strings * (double)A->n_cols * 4.0 > 4.0e18) return PCT_ERANGE;
    return PCT_OK;
}

SapArgs make_args(const pct_csr *A, const pct_sap *p, char *ws, const SapLayout &L) {
    SapArgs a;
    a.m = A->n_rows;
    a.nnz = A->nnz;
    a.n = A->n_cols;
    a.M = p->n_strings;
    a.row_ptr = A->row_ptr_dev;
    a.cols = A->cols_dev;
    a.vals = A->vals_dev;
    a.b = A->b_dev;
    a.order = p->order_dev;
    a.coef = (float *)(ws + L.coef_off);
    a.status = (int32_t *)ws;
    return a;
}

// Largest dynamic LDS of one workgroup on the current device.
size_t lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    return v > 0 ? (size_t)v : 0;
}

template <typename VT>
pct_status launch_strings(const SapArgs &a, const float *x, float *Y, hipStream_t s) {
    const size_t bytes = (size_t)a.n * sizeof(float);
    if (bytes <= lds_limit()) {
        if (hipFuncSetAttribute((const void *)k_sap_string<VT, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes) != hipSuccess)
            return PCT_EHIP;
        hipLaunchKernelGGL((k_sap_string<VT, true>), dim3((unsigned)a.M), dim3(64), bytes, s, a, x, Y);
    } else {
        hipLaunchKernelGGL((k_sap_string<VT, false>), dim3((unsigned)a.M), dim3(64), 0, s, a, x, Y);
    }
    return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
}

}  // namespace
}  // namespace pct

using namespace pct;

extern "C" {

size_t pct_sap_workspace_bytes(const pct_csr *A, const pct_sap *p) {
    if (check_sap(A, p) != PCT_OK) return 0;
    return sap_layout(A->n_rows, A->n_cols, p->n_strings).total;
}

pct_status pct_sap_prepare(const pct_csr *A, const pct_sap *p, void *ws_dev, size_t ws_bytes, void *stream) {
    const pct_status st = check_sap(A, p);
    if (st != PCT_OK) return st;
    const SapLayout L = sap_layout(A->n_rows, A->n_cols, p->n_strings);
    if (!ws_dev || ws_bytes < L.total) return PCT_EWORKSPACE;
    if (p->n_strings > (1 << 30)) return PCT_ERANGE;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)ws_dev;
    const SapArgs a = make_args(A, p, ws, L);
    hipLaunchKernelGGL(k_sap_clear_status, dim3(1), dim3(64), 0, s, a.status);
    // weights in FP64 (uniform: 1/M)
    const int32_t M = p->n_strings;
    double *w = (double *)(ws + L.w_off);
    if (p->weights) {
        if (hipMemcpyAsync(w, p->weights, (size_t)M * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
            return PCT_EHIP;
    } else {
        hipLaunchKernelGGL(k_sap_uniform, dim3((unsigned)((M + 255) / 256)), dim3(256), 0, s, w, M);
    }
    if (A->n_rows > 0) {
        const int64_t blocks64 = (A->n_rows + SAP_WAVES_PREP - 1) / SAP_WAVES_PREP;
        const unsigned blocks = (unsigned)(blocks64 < 65536 ? blocks64 : 65536);
        if (A->val_dtype == PCT_F16)
            hipLaunchKernelGGL((k_sap_prepare<__half>), dim3(blocks), dim3(64 * SAP_WAVES_PREP), 0, s, a, p->relax);
        else
            hipLaunchKernelGGL((k_sap_prepare<float>), dim3(blocks), dim3(64 * SAP_WAVES_PREP), 0, s, a, p->relax);
    }
    return hipGetLastError() == hipSuccess ? PCT_OK : PCT_EHIP;
}

pct_status pct_sap_iterate(const pct_csr *A, const pct_sap *p, float *x_dev, int32_t n_iter, void *ws_dev,
                           size_t ws_bytes, void *stream) {
    const pct_status st = check_sap(A, p);
    if (st != PCT_OK) return st;
    if (n_iter < 0 || !x_dev) return PCT_EINVAL;
    const SapLayout L = sap_layout(A->n_rows, A->n_cols, p->n_strings);
    if (!ws_dev || ws_bytes < L.total) return PCT_EWORKSPACE;
    if (p->n_strings > (1 << 30)) return PCT_ERANGE;
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)ws_dev;
    const SapArgs a = make_args(A, p, ws, L);
    float *Y = (float *)(ws + L.y_off);
    const double *w = (const double *)(ws + L.w_off);
    const unsigned avg_blocks = (unsigned)((A->n_cols + 255) / 256);
    for (int32_t it = 0; it < n_iter; ++it) {
        const pct_status ls = A->val_dtype == PCT_F16 ? launch_strings<__half>(a, x_dev, Y, s)
                                                      : launch_strings<float>(a, x_dev, Y, s);
        if (ls != PCT_OK) return ls;
        hipLaunchKernelGGL(k_sap_average, dim3(avg_blocks), dim3(256), 0, s, Y, w, p->n_strings, A->n_cols, x_dev);
        if (hipGetLastError() != hipSuccess) return PCT_EHIP;
    }
    return PCT_OK;
}

}  // extern "C"

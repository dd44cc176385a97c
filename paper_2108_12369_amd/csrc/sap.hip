// sap.hip -- string-averaging projections (SAP, Sec. II-D) on a CSR system A x = b
// (see include/pct.h for the method and the arithmetic).
//
//   pct_sap_prepare : k_sap_prepare   one wavefront per row: checks its bounds and
//                                     columns, coefficient lambda / ||a_i||^2 (FP64 sum),
//                                     negated for a row that holds a column twice (found
//                                     with a column bitmap in LDS, or a hash table when
//                                     n is large)
//   pct_sap_iterate : k_sap_string    one wavefront per string, y in LDS (when n floats
//                                     fit): y = x_k, then the relaxed projection of every
//                                     row of the string in order; y_t to the workspace
//                     k_sap_string_ws one workgroup of two wavefronts per string, y in the
//                                     workspace: one wave loads the rows, the other
//                                     projects them
//                     k_sap_average   x_{k+1}[j] = sum_t w_t y_t[j] in FP64, t in order
//
// A string is a chain of dependent row updates, so the parallelism is the number of
// strings; one wavefront walks a row's entries 64 at a time.
//
// LDS iterate: the rows' metadata is loaded 64 rows at a time (one row per lane) and the
// first 384 entries of the next four rows are always in flight, so the wave waits on the
// latency of HBM only once per several rows.  With one wave on its SIMD, every issued
// instruction costs the wave its full issue slot, so a row is projected with only as many
// chunks of 64 entries as it spans (a uniform branch on its length picks the body).
//
// Workspace iterate: each row update ends with a wait for its writes to y, and the
// vector-memory counter retires in issue order, so that wait would also drain any row
// loads in flight.  The loads therefore go to a second wavefront, which keeps two rows
// in flight and stages each row (768 entries, values as binary32) in one of two LDS
// slots; the two waves meet at a workgroup barrier once per row.  A row whose columns
// are distinct (the prepare pass marks the others) is written back with plain stores,
// which stay in the XCD's L2 for the next row's gathers; global atomic adds would not.
// The staged entries' gathers and stores go through a buffer resource over y: an entry
// past the row gets an offset outside it (the load returns 0, the store is dropped), so
// each chunk is one instruction with no branch around it.
#include "../../include/pct.h"
#include "pct_device.h"
#include "pct_wave.h"

#include <hip/hip_fp16.h>
#include <math.h>
#include <string.h>

namespace pct {
namespace {

constexpr int SAP_WAVES_PREP = 4;   // waves per block of k_sap_prepare
constexpr int SAP_HASH_BITS = 11;   // per-wave column table of k_sap_prepare: 2048 slots
constexpr int SAP_HASH = 1 << SAP_HASH_BITS;
// Ring of rows in flight: D rows ahead, the first PF chunks of 64 entries of each.  The
// LDS iterate takes short rows from a long ring; the workspace iterate (large grids, long
// curved rows) takes longer rows from a shorter ring.
template <bool LDS> struct Ring { static constexpr int D = 4, PF = 6; };
template <> struct Ring<false> { static constexpr int D = 2, PF = 12; };

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

// A stored value as loaded (binary32, or the 16 bits of a binary16 in a 32-bit register),
// widened only where it is used: converting, or packing two halves into one register,
// right after the load would make the wave wait for it there.
template <typename VT> struct RawOf { using T = float; };
template <> struct RawOf<__half> { using T = uint32_t; };
template <typename VT> __device__ __forceinline__ typename RawOf<VT>::T raw_at(const void *v, int64_t e);
template <> __device__ __forceinline__ float raw_at<float>(const void *v, int64_t e) { return ((const float *)v)[e]; }
template <> __device__ __forceinline__ uint32_t raw_at<__half>(const void *v, int64_t e) {
    return ((const unsigned short *)v)[e];
}
__device__ __forceinline__ float widen(float r) { return r; }
__device__ __forceinline__ float widen(uint32_t r) { return __half2float(__ushort_as_half((unsigned short)r)); }

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

// Enters column c of the row tagged `tag` in a wave's open-addressing table (slots hold
// tag << 32 | column; a slot with another tag is free).  True if the row already holds c,
// or if no free slot was found.
__device__ __forceinline__ bool seen_before(unsigned long long *tab, uint32_t tag, int32_t c) {
    const unsigned long long key = ((unsigned long long)tag << 32) | (uint32_t)c;
    uint32_t h = ((uint32_t)c * 2654435761u) >> (32 - SAP_HASH_BITS);
    for (int step = 0; step < SAP_HASH; ++step) {
        unsigned long long cur = tab[h];
        if ((uint32_t)(cur >> 32) != tag) {
            const unsigned long long prev = atomicCAS(&tab[h], cur, key);
            if (prev == cur) return false;   // claimed
            cur = prev;                      // another lane of this row took it
        }
        if (cur == key) return true;
        h = (h + 1) & (SAP_HASH - 1);
    }
    return true;
}

// One wavefront per row: bounds and columns checked, coefficient lambda / ||a_i||^2 in
// binary64, the norm of the row as a vector of R^n (entries sharing a column summed into
// one component).  A row that holds some column more than once (a curved path can
// re-enter a voxel), or is too long for the column table, gets its coefficient negated:
// the workspace iterate then adds its updates atomically instead of storing them.
// BITS: the repeats are found with a bitmap of the n columns per wave in dynamic LDS
// (one atomic OR per entry, then the row's words cleared) instead of the hash table.
template <typename VT, bool BITS>
__global__ __launch_bounds__(64 * SAP_WAVES_PREP) void k_sap_prepare(SapArgs a, float relax) {
    extern __shared__ uint32_t bitmaps[];
    const int lane = threadIdx.x & 63;
    unsigned long long *tab = nullptr;
    uint32_t *bm = nullptr;
    if constexpr (BITS) {
        const uint32_t words = ((uint32_t)a.n + 31u) / 32u;
        bm = bitmaps + (size_t)(threadIdx.x >> 6) * words;
        for (uint32_t j = lane; j < words; j += 64) bm[j] = 0u;
    } else {
        __shared__ unsigned long long tabs[SAP_WAVES_PREP][SAP_HASH];
        tab = tabs[threadIdx.x >> 6];
        for (int j = lane; j < SAP_HASH; j += 64) tab[j] = ~0ull;   // tag 0xffffffff: never a row's
    }
    const int64_t wid = (int64_t)blockIdx.x * SAP_WAVES_PREP + (threadIdx.x >> 6);
    const int64_t nw = (int64_t)gridDim.x * SAP_WAVES_PREP;
    uint32_t tag = 0;
    for (int64_t i = wid; i < a.m; i += nw, ++tag) {
        const int64_t beg = a.row_ptr[i], end = a.row_ptr[i + 1];
        bool ok = beg >= 0 && end >= beg && end <= a.nnz;
        const bool hashable = BITS || (ok && end - beg <= SAP_HASH / 2);
        bool dup = false;
        double nrm = 0.0;
        if (ok) {
            // eight chunks of 64 entries loaded before any is used, so that a row's loads
            // overlap (the wave has little else to hide their latency); a row of at most
            // 512 entries is cleared from the columns still in registers
            constexpr int U = 8;
            const bool one_pass = end - beg <= 64 * U;   // uniform
            int32_t cu[U];
            float vu[U];
            for (int64_t e0 = beg + lane; e0 < end; e0 += 64 * U) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t e = e0 + u * 64;
                    cu[u] = e < end ? a.cols[e] : 0;
                    vu[u] = e < end ? val_at<VT>(a.vals, e) : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (e0 + u * 64 < end) {
                        const int32_t c = cu[u];
                        const bool okc = (uint32_t)c < (uint32_t)a.n;
                        ok = ok && okc;
                        const double v = (double)vu[u];
                        nrm = fma(v, v, nrm);
                        if constexpr (BITS) {
                            if (okc) {
                                const uint32_t bit = 1u << ((uint32_t)c & 31u);
                                if (atomicOr(bm + ((uint32_t)c >> 5), bit) & bit) dup = true;
                            }
                        } else {
                            if (hashable && seen_before(tab, tag, c)) dup = true;
                        }
                    }
                }
            }
            if constexpr (BITS) {
                // the row's words back to zero (the wave's LDS accesses are in order)
                __builtin_amdgcn_wave_barrier();
                if (one_pass) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        if (beg + lane + u * 64 < end && (uint32_t)cu[u] < (uint32_t)a.n) bm[(uint32_t)cu[u] >> 5] = 0u;
                } else {
                    for (int64_t e = beg + lane; e < end; e += 64) {
                        const int32_t c = a.cols[e];
                        if ((uint32_t)c < (uint32_t)a.n) bm[(uint32_t)c >> 5] = 0u;
                    }
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        const bool all_ok = __builtin_amdgcn_ballot_w64(!ok) == 0;
        const bool repeats = !hashable || __builtin_amdgcn_ballot_w64(dup) != 0;
        if (repeats && all_ok) {
            // ||a_i||^2 of the row as a vector: entries that share a column add into one
            // component, so the sum over entries e of v_e * (sum of the values of e's
            // column), which counts each column's (sum of values)^2 once.  Every lane
            // compares its entries with all of the row's (loads of a uniform index),
            // quadratic in the row length; rows that repeat a column are few.
            nrm = 0.0;
            for (int64_t e0 = beg; e0 < end; e0 += 64) {
                const int64_t e = e0 + lane;
                const int32_t ce = e < end ? a.cols[e] : -1;
                const double ve = e < end ? (double)val_at<VT>(a.vals, e) : 0.0;
                double s = 0.0;
                for (int64_t f = beg; f < end; ++f) {
                    const int32_t cf = a.cols[f];
                    const double vf = (double)val_at<VT>(a.vals, f);
                    s += cf == ce ? vf : 0.0;
                }
                nrm = fma(ve, s, nrm);
            }
        }
        nrm = wave_sum(nrm);
        if (lane == 0) {
            const float cf = (all_ok && nrm > 0.0) ? (float)((double)relax / nrm) : 0.0f;
            a.coef[i] = repeats ? -cf : cf;
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

// The workspace copy of y, which only the string's own workgroup reads and writes
// (workgroup scope).
__device__ __forceinline__ float ws_load(float *y, int32_t c) {
    return __hip_atomic_load(y + c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Workspace update of a row whose columns are distinct: y[c] = y_c + alpha v, the same
// binary32 arithmetic as the atomic add, as a store (it stays in this XCD's L2, where the
// next gathers find it; an atomic add makes them go further).
__device__ __forceinline__ void ws_put(float *y, int32_t c, float v) {
    __hip_atomic_store(y + c, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Workspace update of a row that holds some column twice.
__device__ __forceinline__ void ws_add(float *y, int32_t c, float v) { unsafeAtomicAdd(y + c, v); }

// Workspace iterate: the wave's writes (performed in L2) are complete before its next
// loads (which read L2).  The fence keeps the compiler from moving memory accesses across.
__device__ __forceinline__ void ws_settle() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// First PF chunks of a row's entries.  The loads are unconditional (an index past the
// row reads a valid entry of the arrays, nnz > 0) so that nothing waits for them here;
// whether an entry belongs to the row is decided where it is used.
template <typename VT, int PF>
__device__ __forceinline__ void fetch_chunks(const SapArgs &a, const RowMeta &r, int lane, int32_t (&c)[PF],
                                             typename RawOf<VT>::T (&v)[PF]) {
    // a uniform base (the row's first entry, or the last entry of the arrays for an empty
    // row at their end) and 32-bit lane offsets clamped to the arrays' end
    const int64_t last = a.nnz - 1;
    const int64_t base = r.beg < last ? r.beg : last;
    const int64_t room = last - base;
    const uint32_t lim = room < 0x7fffffff ? (uint32_t)room : 0x7fffffffu;
    const int32_t *cb = a.cols + base;
    const void *vb = (const char *)a.vals + base * (int64_t)sizeof(VT);
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const uint32_t o = (uint32_t)(k * 64 + lane) < lim ? (uint32_t)(k * 64 + lane) : lim;
        c[k] = cb[o];
        v[k] = raw_at<VT>(vb, (int64_t)o);
    }
}

// One row of a string projected onto y in LDS with the first NC of the PF prefetched
// chunks in cc / cv (the row holds no entry past them unless NC = PF); the adds are LDS
// atomics, since the entries of a row may share a voxel.
template <typename VT, int PF, int NC>
__device__ __forceinline__ void project_chunks(const SapArgs &a, float *y, const RowMeta &r, uint32_t len,
                                               const int32_t (&cc)[PF], const typename RawOf<VT>::T (&cv)[PF],
                                               int lane) {
    const uint32_t n = (uint32_t)a.n;
    bool ok[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) ok[k] = (uint32_t)(k * 64 + lane) < len && (uint32_t)cc[k] < n;
    // all gathers in flight before the first use; an entry past the row or with a bad
    // column reads y[0] and counts 0
    float yv[NC];
#pragma unroll
    for (int k = 0; k < NC; ++k) yv[k] = y[ok[k] ? cc[k] : 0];
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < NC; ++k) acc = fma((double)(ok[k] ? widen(cv[k]) : 0.0f), (double)yv[k], acc);
    const bool tail = NC == PF && len > (uint32_t)(PF * 64);   // uniform
    if (tail) {
        for (int64_t e = r.beg + PF * 64 + lane; e < r.end; e += 64) {
            const int32_t c = a.cols[e];
            const bool okc = (uint32_t)c < n;
            const float yc = y[okc ? c : 0];
            acc = fma((double)(okc ? val_at<VT>(a.vals, e) : 0.0f), (double)yc, acc);
        }
    }
    const double dot = wave_sum(acc);
    const float alpha = (float)(((double)r.b - dot) * (double)fabsf(r.coef));
    // no branch: an entry that is not the row's adds 0 to its lane's spare slot past y
#pragma unroll
    for (int k = 0; k < NC; ++k)
        atomicAdd(y + (ok[k] ? (uint32_t)cc[k] : n + (uint32_t)lane), ok[k] ? alpha * widen(cv[k]) : 0.0f);
    if (tail) {
        for (int64_t e = r.beg + PF * 64 + lane; e < r.end; e += 64) {
            const int32_t c = a.cols[e];
            if ((uint32_t)c < n) atomicAdd(y + c, alpha * val_at<VT>(a.vals, e));
        }
    }
}

template <typename VT, int PF>
__device__ __forceinline__ void project_row(const SapArgs &a, float *y, const RowMeta &r, const int32_t (&cc)[PF],
                                            const typename RawOf<VT>::T (&cv)[PF], int lane) {
    static_assert(PF == 6, "one body per chunk count");
    if (r.coef == 0.0f) return;
    const int64_t len64 = r.end - r.beg;   // a row is shorter than 2^31 entries
    const uint32_t len = len64 < 0x7fffffff ? (uint32_t)len64 : 0x7fffffffu;
    switch ((len + 63) / 64) {   // chunks the row spans (a row with coefficient != 0 has one)
    case 0: break;
    case 1: project_chunks<VT, PF, 1>(a, y, r, len, cc, cv, lane); break;
    case 2: project_chunks<VT, PF, 2>(a, y, r, len, cc, cv, lane); break;
    case 3: project_chunks<VT, PF, 3>(a, y, r, len, cc, cv, lane); break;
    case 4: project_chunks<VT, PF, 4>(a, y, r, len, cc, cv, lane); break;
    case 5: project_chunks<VT, PF, 5>(a, y, r, len, cc, cv, lane); break;
    default: project_chunks<VT, PF, PF>(a, y, r, len, cc, cv, lane); break;
    }
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

template <typename VT>
__global__ __launch_bounds__(64) void k_sap_string(SapArgs a, const float *x, float *Y) {
    extern __shared__ float ys[];
    constexpr int D = Ring<true>::D, PF = Ring<true>::PF;
    const int lane = threadIdx.x;
    const int t = blockIdx.x;
    const int n = a.n;
    float *yg = Y + (size_t)t * (size_t)n;
    float *y = ys;
    for (int j = lane; j < n; j += 64) y[j] = x[j];
    __syncthreads();
    if (a.nnz == 0) {   // every row empty: nothing to load (and no entry to clamp to)
        for (int j = lane; j < n; j += 64) yg[j] = ys[j];
        return;
    }

    // The string's positions go in batches of 64 whose metadata the lanes hold (this
    // batch in A, the next one in B).  Slot j of the ring holds the first PF chunks of
    // the row at position j (mod D); a slot is refilled with the row D positions on as
    // soon as its row is projected, so the loads of D rows are always in flight.
    const int64_t s0 = (int64_t)t * a.m / a.M, s1 = (int64_t)(t + 1) * a.m / a.M;
    LaneMeta A = lane_meta(a, s0, s1, lane), B = lane_meta(a, s0 + 64, s1, lane);
    int32_t cq[D][PF];
    typename RawOf<VT>::T vq[D][PF];
#pragma unroll
    for (int j = 0; j < D; ++j) {
        fetch_chunks<VT, PF>(a, meta_at(A, j), lane, cq[j], vq[j]);
        __builtin_amdgcn_sched_barrier(0);   // slots filled in order
    }
    static_assert(64 % D == 0, "whole ring turns per batch");
    for (int64_t sb = s0; sb < s1; sb += 64) {
        // the position D on is in this batch, except in the batch's last ring turn
        for (int j0 = 0; j0 < 64 - D; j0 += D) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                project_row<VT, PF>(a, y, meta_at(A, j0 + j), cq[j], vq[j], lane);
                fetch_chunks<VT, PF>(a, meta_at(A, j0 + j + D), lane, cq[j], vq[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < D; ++j) {
            project_row<VT, PF>(a, y, meta_at(A, 64 - D + j), cq[j], vq[j], lane);
            fetch_chunks<VT, PF>(a, meta_at(B, j), lane, cq[j], vq[j]);
        }
        A = B;
        B = lane_meta(a, sb + 128, s1, lane);
    }
    __syncthreads();
    for (int j = lane; j < n; j += 64) yg[j] = ys[j];
}

// Buffer access to a string's y (n binary32): an offset at or past 4 n bytes is outside
// the resource (n < 2^29, checked on the host, so Y_OUT always is).  Cache policy as the
// workgroup-scope accesses above.
constexpr uint32_t Y_OUT = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t y_rsrc(float *y, int32_t n) {
    return __builtin_amdgcn_make_buffer_rsrc(y, (short)0, n * 4, 0x00020000);
}
__device__ __forceinline__ float yb_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 1));
}
__device__ __forceinline__ void yb_store(__amdgpu_buffer_rsrc_t r, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 1);
}

// Barrier between the two waves of k_sap_string_ws: their LDS accesses before it happen
// before those after it (lgkmcnt(0), s_barrier); global loads stay in flight.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename VT>
__global__ __launch_bounds__(128) void k_sap_string_ws(SapArgs a, const float *x, float *Y) {
    constexpr int D = Ring<false>::D, PF = Ring<false>::PF, SLOT = PF * 64;
    __shared__ int32_t sc[2][SLOT];
    __shared__ float sv[2][SLOT];
    __shared__ int64_t sbeg[2], send[2];
    __shared__ float sb[2], scoef[2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int t = blockIdx.x;
    const int n = a.n;
    float *y = Y + (size_t)t * (size_t)n;
    for (int j = threadIdx.x; j < n; j += 128) y[j] = x[j];
    __syncthreads();   // (global and LDS) the copy is in L2 before the first gathers
    if (a.nnz == 0) return;   // every row empty (both waves leave here)

    const int64_t s0 = (int64_t)t * a.m / a.M, s1 = (int64_t)(t + 1) * a.m / a.M;
    const int64_t L = s1 - s0;
    // Step k: the loader stages position k in slot k & 1 while the projector projects
    // position k - 1 from slot (k - 1) & 1.  Both waves take the same number of steps
    // (L + 1 rounded up to a multiple of D) and the barrier of each; positions past the
    // string are empty rows (coefficient 0), so no step depends on a row's contents.
    static_assert(D % 2 == 0 && 64 % D == 0, "ring depth");
    const int64_t steps = (L + D) / D * D;
    if (wave == 1) {
        // loader: ring of D rows whose first SLOT entries are in flight
        LaneMeta A = lane_meta(a, s0, s1, lane), B = lane_meta(a, s0 + 64, s1, lane);
        int32_t cq[D][PF];
        typename RawOf<VT>::T vq[D][PF];
        // the slots are filled in order (the scheduler may not interleave them), so a
        // slot's loads are always older than those of the slots after it
#pragma unroll
        for (int j = 0; j < D; ++j) {
            fetch_chunks<VT, PF>(a, meta_at(A, j), lane, cq[j], vq[j]);
            __builtin_amdgcn_sched_barrier(0);
        }
        for (int64_t sb0 = 0; sb0 < steps; sb0 += 64) {
            const int jn = steps - sb0 < 64 ? (int)(steps - sb0) : 64;
            for (int j0 = 0; j0 < jn; j0 += D) {
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const int slot = j & 1;   // = k & 1, as sb0 and j0 are even
                    const RowMeta r = meta_at(A, j0 + j);
#pragma unroll
                    for (int q = 0; q < PF; ++q) {
                        sc[slot][q * 64 + lane] = cq[j][q];
                        sv[slot][q * 64 + lane] = widen(vq[j][q]);
                    }
                    if (lane == 0) {
                        sbeg[slot] = r.beg;
                        send[slot] = r.end;
                        sb[slot] = r.b;
                        scoef[slot] = r.coef;
                    }
                    const int nx = j0 + j + D;
                    const RowMeta mn = nx < 64 ? meta_at(A, nx) : meta_at(B, nx - 64);
                    fetch_chunks<VT, PF>(a, mn, lane, cq[j], vq[j]);
                    lds_barrier();
                }
            }
            A = B;
            B = lane_meta(a, s0 + sb0 + 128, s1, lane);
        }
    } else {
        // projector
        const uint32_t nu = (uint32_t)n;
        const __amdgpu_buffer_rsrc_t yr = y_rsrc(y, n);
        for (int64_t k = 0; k < steps; ++k) {
            if (k > 0) {
                const int slot = (int)((k - 1) & 1);
                const float cf = scoef[slot];
                if (cf != 0.0f) {
                    const bool repeats = cf < 0.0f;   // some column twice: atomic adds
                    const float coef = fabsf(cf);
                    const int64_t beg = sbeg[slot], end = send[slot];
                    int32_t cc[PF];
                    float cv[PF], yv[PF];
                    bool ok[PF];
#pragma unroll
                    for (int q = 0; q < PF; ++q) {
                        cc[q] = sc[slot][q * 64 + lane];
                        cv[q] = sv[slot][q * 64 + lane];
                        ok[q] = beg + q * 64 + lane < end && (uint32_t)cc[q] < nu;
                    }
#pragma unroll
                    for (int q = 0; q < PF; ++q) yv[q] = yb_load(yr, ok[q] ? (uint32_t)cc[q] * 4u : Y_OUT);
                    double acc = 0.0;
#pragma unroll
                    for (int q = 0; q < PF; ++q) acc = fma(ok[q] ? (double)cv[q] : 0.0, (double)yv[q], acc);
                    for (int64_t e = beg + SLOT + lane; e < end; e += 64) {
                        const int32_t c = a.cols[e];
                        const bool okc = (uint32_t)c < nu;
                        const float yc = ws_load(y, okc ? c : 0);
                        acc = fma(okc ? (double)val_at<VT>(a.vals, e) : 0.0, (double)yc, acc);
                    }
                    const double dot = wave_sum(acc);
                    const float alpha = (float)(((double)sb[slot] - dot) * (double)coef);
                    if (repeats) {
#pragma unroll
                        for (int q = 0; q < PF; ++q)
                            if (ok[q]) ws_add(y, cc[q], alpha * cv[q]);
                        for (int64_t e = beg + SLOT + lane; e < end; e += 64) {
                            const int32_t c = a.cols[e];
                            if ((uint32_t)c < nu) ws_add(y, c, alpha * val_at<VT>(a.vals, e));
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < PF; ++q)
                            yb_store(yr, ok[q] ? (uint32_t)cc[q] * 4u : Y_OUT, yv[q] + alpha * cv[q]);
                        for (int64_t e = beg + SLOT + lane; e < end; e += 64) {
                            const int32_t c = a.cols[e];
                            if ((uint32_t)c < nu) ws_put(y, c, ws_load(y, c) + alpha * val_at<VT>(a.vals, e));
                        }
                    }
                    // the next row's gathers must see these adds
                    ws_settle();
                }
            }
            lds_barrier();
        }
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
    if (A->n_cols >= (1 << 29)) return PCT_ERANGE;   // byte offsets into one string's y
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
    // y and one spare slot per lane (the target of the adds of entries past a row)
    const size_t bytes = ((size_t)a.n + 64) * sizeof(float);
    if (bytes <= lds_limit()) {
        if (hipFuncSetAttribute((const void *)k_sap_string<VT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes) != hipSuccess)
            return PCT_EHIP;
        hipLaunchKernelGGL((k_sap_string<VT>), dim3((unsigned)a.M), dim3(64), bytes, s, a, x, Y);
    } else {
        hipLaunchKernelGGL((k_sap_string_ws<VT>), dim3((unsigned)a.M), dim3(128), 0, s, a, x, Y);
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
        // a column bitmap per wave when two blocks of them fit a CU's LDS, else the hash
        const size_t bm_bytes = (size_t)SAP_WAVES_PREP * (((size_t)A->n_cols + 31) / 32) * sizeof(uint32_t);
        const bool bits = 2 * bm_bytes <= lds_limit();
        if (bits) {
            const void *k = A->val_dtype == PCT_F16 ? (const void *)k_sap_prepare<__half, true>
                                                    : (const void *)k_sap_prepare<float, true>;
            if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bm_bytes) != hipSuccess)
                return PCT_EHIP;
            if (A->val_dtype == PCT_F16)
                hipLaunchKernelGGL((k_sap_prepare<__half, true>), dim3(blocks), dim3(64 * SAP_WAVES_PREP), bm_bytes, s,
                                   a, p->relax);
            else
                hipLaunchKernelGGL((k_sap_prepare<float, true>), dim3(blocks), dim3(64 * SAP_WAVES_PREP), bm_bytes, s,
                                   a, p->relax);
        } else if (A->val_dtype == PCT_F16) {
            hipLaunchKernelGGL((k_sap_prepare<__half, false>), dim3(blocks), dim3(64 * SAP_WAVES_PREP), 0, s, a,
                               p->relax);
        } else {
            hipLaunchKernelGGL((k_sap_prepare<float, false>), dim3(blocks), dim3(64 * SAP_WAVES_PREP), 0, s, a,
                               p->relax);
        }
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

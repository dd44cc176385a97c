// pct_wave.h -- wave-cooperative emit of CSR rows (gfx950, wave64).
//
// One wavefront walks one proton path at a time.  The path is cut into "items":
//   - cells of a straight ray (the part of the ray between two consecutive faces of its
//     dominant axis, the axis with the most crossings per unit length), for the ray
//     before the entry point, the ray after the exit point, or the whole path of a
//     straight proton;
//   - chords between consecutive samples of the cubic spline.
// Each lane takes K consecutive items.  A first pass over them finds the voxel index at
// every item end (FP64 positions, floor) and counts the face crossings; a wave prefix
// sum of the crossing counts places every lane's entries in the row; a second pass
// orders the crossings inside each item, cuts it into per-voxel pieces (FP32 lengths)
// and writes the entries that close inside the lane.  The entry that is open when a
// lane starts (it began in an earlier lane) gets its length from a segmented scan over
// the lanes and is written by the lane that closes it.  The stores of one row are one
// contiguous range, written by the whole wave.
//
// Consecutive items share end points, so the voxel at the end of an item is the voxel
// at the start of the next and the row has exactly 1 + (number of crossings) entries,
// the same number the count pass finds.  Paths whose spline may leave the grid box are
// walked by the per-lane code (trace_row) instead.
#pragma once

#include "pct_device.h"

namespace pct {

constexpr int WAVE = 64;
constexpr int BATCH = 16;   // rows prepared per wave at a time (one per lane)

// A straight ray prepared for the cell walk (uniform over the wave).
template <typename R>
struct RayW {
    R A[3], D[3], invD[3];
    R lo, hi, Dn;
    int is[3], ie[3];
    int dom, sdom, ncell;
    // the dominant axis's values, kept apart so that no array is indexed at run time
    R a_dom, inv_dom, o_dom, h_dom;
    int is_dom;
};

// Per-row description of the path, written by the count pass (one lane per row) into
// the workspace and read by the emit pass with uniform (scalar) loads: the prepared
// rays (the whole straight path, or the rays before the entry and after the exit) and
// the spline's power basis.
template <typename R>
struct RowW {
    int32_t kind;       // 0: no entry, 1: one ray, 2: ray + spline + ray, 3: per-lane walk
    int32_t N;          // spline chords
    RayW<R> ray[2];     // ray[0].A is the entry point P0, ray[1].A the exit point P1 (kind 2)
    R c1[3], c2[3], c3[3];   // spline power basis, origin P0
    R invN;
    double bfac;        // WEPL noise factor 1 + r z
};

template <typename R, int DIM>
__device__ __forceinline__ void ray_prepare(const JobDev &J, const R A[3], const R D[3], R lo, R hi,
                                            RayW<R> &r) {
    R dn2 = R(0), best = R(-1);
    r.dom = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r.A[d] = A[d];
        r.D[d] = D[d];
        r.invD[d] = R(0);
        r.is[d] = 0;
        r.ie[d] = 0;
        if (d < DIM) {
            dn2 += D[d] * D[d];
            r.invD[d] = (D[d] != R(0)) ? R(1) / D[d] : R(0);
            const R P = A[d] + lo * D[d];
            const R E = A[d] + hi * D[d];
            r.is[d] = vox_index<R>(P, J.o[d], J.invh[d], J.n[d]);
            r.ie[d] = vox_index<R>(E, J.o[d], J.invh[d], J.n[d]);
            const R rate = (D[d] < R(0) ? -D[d] : D[d]) * R(J.invh[d]);
            if (rate > best) {
                best = rate;
                r.dom = d;
            }
        }
    }
    r.lo = lo;
    r.hi = hi;
    r.Dn = r_sqrt<R>(dn2);
    int dd = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        if (d == r.dom) {
            dd = r.ie[d] - r.is[d];
            r.is_dom = r.is[d];
            r.a_dom = A[d];
            r.inv_dom = r.invD[d];
            r.o_dom = R(J.o[d]);
            r.h_dom = R(J.h[d]);
        }
    }
    r.sdom = dd >= 0 ? 1 : -1;
    r.ncell = (lo < hi) ? abs(dd) + 1 : 0;   // no cell when the ray misses the box
}

// Parameter of the dominant-axis face between cell m-1 and cell m (1 <= m < ncell).
template <typename R>
__device__ __forceinline__ R ray_bound(const JobDev &J, const RayW<R> &r, int m) {
    const int k = r.is_dom + (m - 1) * r.sdom + (r.sdom > 0 ? 1 : 0);
    const R plane = r.o_dom + R(k) * r.h_dom;
    return (plane - r.a_dom) * r.inv_dom;
}

// Voxel at the start of cell m (its parameter lam given).
template <typename R, int DIM>
__device__ __forceinline__ void ray_index(const JobDev &J, const RayW<R> &r, int m, R lam, int I[3]) {
    if (m == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) I[d] = r.is[d];
        return;
    }
    if (m == r.ncell) {
#pragma unroll
        for (int d = 0; d < 3; ++d) I[d] = r.ie[d];
        return;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < DIM) {
            if (d == r.dom) {
                I[d] = r.is_dom + m * r.sdom;
            } else {
                // kept between the end voxels so that the steps per axis add up to
                // |ie - is| whatever the rounding of the boundary parameters
                const int v = vox_index<R>(r.A[d] + lam * r.D[d], J.o[d], J.invh[d], J.n[d]);
                const int lo = r.is[d] < r.ie[d] ? r.is[d] : r.ie[d];
                const int hi = r.is[d] < r.ie[d] ? r.ie[d] : r.is[d];
                I[d] = v < lo ? lo : (v > hi ? hi : v);
            }
        } else {
            I[d] = 0;
        }
    }
}

template <typename R>
__device__ __forceinline__ R ray_lam(const JobDev &J, const RayW<R> &r, int m) {
    return (m == 0) ? r.lo : (m == r.ncell) ? r.hi : ray_bound<R>(J, r, m);
}

// ------------------------------------------------------------------ wave helpers
template <typename T>
__device__ __forceinline__ T shfl_up_t(T v, int off) {
    return __shfl_up(v, (unsigned)off, WAVE);
}

// Inclusive add-scan over the wavefront with DPP: shifts by 1, 2, 4, 8 inside each row
// of 16 lanes, then the last lane of row 0 / rows 0-1 is added to the rows after it.
__device__ __forceinline__ int wave_incl_scan(int v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31
    return v;
}

__device__ __forceinline__ int wave_excl_scan(int v, int lane, int &total) {
    (void)lane;
    const int s = wave_incl_scan(v);
    total = __builtin_amdgcn_readlane(s, WAVE - 1);
    return s - v;
}

// One step of the segmented scan: a lane without a reset so far takes the value of the
// lane `ctrl` selects and adds it.
template <int CTRL, int ROWMASK, bool BOUND>
__device__ __forceinline__ void seg_step(float &v, int &f) {
    const float vo = __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                                           ROWMASK, 0xf, BOUND));
    const int fo = __builtin_amdgcn_update_dpp(0, f, CTRL, ROWMASK, 0xf, BOUND);
    if (!f) {
        v += vo;
        f = fo;
    }
}

// Inclusive segmented sum: value restarts at lanes with f set.
__device__ __forceinline__ void wave_seg_scan(float &v, int &f) {
    seg_step<0x111, 0xf, true>(v, f);
    seg_step<0x112, 0xf, true>(v, f);
    seg_step<0x114, 0xf, true>(v, f);
    seg_step<0x118, 0xf, true>(v, f);
    seg_step<0x142, 0xa, false>(v, f);
    seg_step<0x143, 0xc, false>(v, f);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Output of one row: entries at row-relative indices [0, len) of the row's slices of
// cols / vals (uniform base pointers, 32-bit offsets); WEPL partial per lane in FP32
// over at most a block's entries, folded into TW once per block.
template <typename TW>
struct RowOut {
    int32_t *cols;
    __half *vh;
    float *vf;
    const float *x;
    int32_t len;
    float wepl;
    TW wacc;
    bool store, half, want_b;

    __device__ __forceinline__ void put(int32_t rel, int32_t col, float l) {
        if (want_b) wepl = fmaf(l, x[col], wepl);
        if (store && rel < len) {
            cols[rel] = col;
            if (half) vh[rel] = __float2half_rn(l);
            else vf[rel] = l;
        }
    }
    __device__ __forceinline__ void fold() {
        wacc += (TW)wepl;
        wepl = 0.f;
    }
};

template <typename R, int DIM>
__device__ __forceinline__ void spline_at(const RowW<R> &w, int j, R out[3]) {
    if (j == 0) {
#pragma unroll
        for (int d = 0; d < 3; ++d) out[d] = w.ray[0].A[d];
        return;
    }
    if (j == w.N) {
#pragma unroll
        for (int d = 0; d < 3; ++d) out[d] = w.ray[1].A[d];
        return;
    }
    const R s = R(j) * w.invN;
#pragma unroll
    for (int d = 0; d < 3; ++d)
        out[d] = (d < DIM) ? r_fma<R>(r_fma<R>(r_fma<R>(w.c3[d], s, w.c2[d]), s, w.c1[d]), s, w.ray[0].A[d]) : R(0);
}

// Voxel of a spline sample.  The row's control-point hull lies in the box, so the floor
// is already in range; the clamp only guards the gather and the stores.
template <typename R, int DIM>
__device__ __forceinline__ void spline_index(const JobDev &J, const R p[3], int I[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int v = (d < DIM) ? (int)vox_floor<R>(p[d], J.o[d], J.invh[d]) : 0;
        I[d] = v < 0 ? 0 : (v > J.n[d] - 1 ? J.n[d] - 1 : v);
    }
}

// Pieces of one item between state (Ip, Pp) and (Ie, Pe): every crossing closes the
// open entry.  Callback close(ok, col, length) receives each closed entry's last piece
// (ok false: no entry in this slot).  The general forms below loop over any number of
// crossings; the fast forms handle at most one crossing per axis without branches.
template <typename R>
struct Walker {
    float head, pend;
    int done;
    int32_t cur;
};

template <typename R, int DIM, class F>
__device__ __forceinline__ void chord_pieces(const JobDev &J, const int Ip[3], const R Pp[3], const int Ie[3],
                                             const R Pe[3], Walker<R> &wk, F &&close) {
    int bud[3] = {0, 0, 0}, st[3] = {0, 0, 0}, tot = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int dd = Ie[d] - Ip[d];
        bud[d] = abs(dd);
        st[d] = dd > 0 ? 1 : -1;
        tot += bud[d];
    }
    R D[3] = {R(0), R(0), R(0)};
    float dn2 = 0.f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        D[d] = Pe[d] - Pp[d];
        const float f = (float)D[d];
        dn2 = fmaf(f, f, dn2);
    }
    const float len = __builtin_amdgcn_sqrtf(dn2);
    if (tot == 0) {
        wk.pend += len;
        return;
    }
    int I[3] = {Ip[0], Ip[1], Ip[2]};
    float lp = 0.f;
    while (tot > 0) {
        int a = -1;
        R na = R(0), da = R(1);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if (bud[d] > 0) {
                const R plane = R(J.o[d]) + R(I[d] + (st[d] > 0 ? 1 : 0)) * R(J.h[d]);
                const R nd = plane - Pp[d];
                const R ad = D[d] < R(0) ? -D[d] : D[d];
                const R an = nd < R(0) ? -nd : nd;
                if (a < 0 || an * da < na * ad) {
                    a = d;
                    na = an;
                    da = ad;
                }
            }
        }
        float lc = (float)na * __builtin_amdgcn_rcpf((float)da);
        lc = lc > lp ? lc : lp;
        lc = lc < 1.f ? lc : 1.f;
        close(true, wk.cur, wk.pend + (lc - lp) * len);
        wk.pend = 0.f;
        lp = lc;
        if (a == 0) { I[0] += st[0]; bud[0] -= 1; }
        else if (a == 1) { I[1] += st[1]; bud[1] -= 1; }
        else { I[2] += st[2]; bud[2] -= 1; }
        --tot;
        wk.cur = col_of<DIM>(J, I);
    }
    wk.pend += (1.f - lp) * len;
}

template <typename R, int DIM, class F>
__device__ __forceinline__ void cell_pieces(const JobDev &J, const RayW<R> &r, const int Ip[3], R lp,
                                            const int Ie[3], R le, Walker<R> &wk, F &&close) {
    int bud[3] = {0, 0, 0}, st[3] = {0, 0, 0}, tot = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int dd = Ie[d] - Ip[d];
        bud[d] = abs(dd);
        st[d] = dd > 0 ? 1 : -1;
        tot += bud[d];
    }
    int I[3] = {Ip[0], Ip[1], Ip[2]};
    while (tot > 0) {
        int a = -1;
        R la = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if (bud[d] > 0) {
                R ld;
                if (d == r.dom) {
                    ld = le;
                } else {
                    const R plane = R(J.o[d]) + R(I[d] + (st[d] > 0 ? 1 : 0)) * R(J.h[d]);
                    ld = (plane - r.A[d]) * r.invD[d];
                }
                if (a < 0 || ld < la) {
                    a = d;
                    la = ld;
                }
            }
        }
        R lc = la > lp ? la : lp;
        lc = lc < le ? lc : le;
        close(true, wk.cur, wk.pend + (float)((lc - lp) * r.Dn));
        wk.pend = 0.f;
        lp = lc;
        if (a == 0) { I[0] += st[0]; bud[0] -= 1; }
        else if (a == 1) { I[1] += st[1]; bud[1] -= 1; }
        else { I[2] += st[2]; bud[2] -= 1; }
        --tot;
        wk.cur = col_of<DIM>(J, I);
    }
    wk.pend += (float)((le - lp) * r.Dn);
}

// ---------------------------------------------------------- branch-free item pieces
// One candidate crossing per axis: ordering key, FP32 parameter, column step.
template <typename R>
struct Cross {
    R kn, kd;       // key = kn / kd (kd > 0); compared cross-multiplied
    float lam;      // parameter of the crossing in the item, FP32
    int32_t dcol;   // column change when it is passed
    bool ok;        // the axis does cross in this item
};

template <typename R>
__device__ __forceinline__ bool cross_before(const Cross<R> &a, const Cross<R> &b) {
    // valid first; then smaller parameter; ties keep the lower axis (callers order a < b)
    return a.ok && (!b.ok || a.kn * b.kd <= b.kn * a.kd);
}

template <typename R>
__device__ __forceinline__ void cswap(Cross<R> &a, Cross<R> &b) {
    if (!cross_before(a, b)) {
        const Cross<R> t = a;
        a = b;
        b = t;
    }
}

template <typename R, int DIM>
__device__ __forceinline__ void sort_cross(Cross<R> c[3]) {
    cswap(c[0], c[1]);
    if (DIM == 3) {
        cswap(c[1], c[2]);
        cswap(c[0], c[1]);
    }
}

template <int DIM>
__device__ __forceinline__ int32_t col_stride(const JobDev &J, int d) {
    return d == 0 ? 1 : (d == 1 ? J.n[0] : J.n[0] * J.n[1]);
}

// Chord from Pp to Pe with at most one crossing per axis.
template <typename R, int DIM, class F>
__device__ __forceinline__ void chord_fast(const JobDev &J, const int Ip[3], const R Pp[3], const int Ie[3],
                                           const R Pe[3], Walker<R> &wk, F &&close) {
    Cross<R> c[3];
    float dn2 = 0.f;
    int tot = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d].ok = false;
        c[d].kn = R(0);
        c[d].kd = R(1);
        c[d].lam = 2.f;
        c[d].dcol = 0;
        if (d < DIM) {
            const R D = Pe[d] - Pp[d];
            const float f = (float)D;
            dn2 = fmaf(f, f, dn2);
            const int dd = Ie[d] - Ip[d];
            const bool up = dd > 0;
            c[d].ok = dd != 0;
            tot += c[d].ok ? 1 : 0;
            const R plane = R(J.o[d]) + R(Ip[d] + (up ? 1 : 0)) * R(J.h[d]);
            const R nd = plane - Pp[d];
            c[d].kn = nd < R(0) ? -nd : nd;
            c[d].kd = D < R(0) ? -D : D;
            c[d].lam = (float)c[d].kn * __builtin_amdgcn_rcpf((float)c[d].kd);
            c[d].dcol = (up ? 1 : -1) * col_stride<DIM>(J, d);
        }
    }
    const float len = __builtin_amdgcn_sqrtf(dn2);
    sort_cross<R, DIM>(c);
    float lp = 0.f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const bool ok = k < tot;
        float lc = c[k].lam > lp ? c[k].lam : lp;
        lc = lc < 1.f ? lc : 1.f;
        close(ok, wk.cur, (k == 0 ? wk.pend : 0.f) + (lc - lp) * len);
        wk.cur += ok ? c[k].dcol : 0;
        lp = ok ? lc : lp;
    }
    wk.pend = (tot == 0 ? wk.pend : 0.f) + (1.f - lp) * len;
}

// Ray cell from parameter lp to le with at most one crossing per axis (the dominant
// axis crosses at le unless this is the ray's last cell).
template <typename R, int DIM, class F>
__device__ __forceinline__ void cell_fast(const JobDev &J, const RayW<R> &r, const int Ip[3], R lp,
                                          const int Ie[3], R le, Walker<R> &wk, F &&close) {
    Cross<R> c[3];
    R lam64[3];
    int tot = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        c[d].ok = false;
        c[d].kn = R(0);
        c[d].kd = R(1);
        c[d].lam = 0.f;
        c[d].dcol = 0;
        lam64[d] = le;
        if (d < DIM) {
            const int dd = Ie[d] - Ip[d];
            const bool up = dd > 0;
            c[d].ok = dd != 0;
            tot += c[d].ok ? 1 : 0;
            R ld = le;
            if (d != r.dom) {
                const R plane = R(J.o[d]) + R(Ip[d] + (up ? 1 : 0)) * R(J.h[d]);
                ld = (plane - r.A[d]) * r.invD[d];
            }
            lam64[d] = ld;
            c[d].kn = ld;   // keys compared directly (kd = 1)
            c[d].dcol = (up ? 1 : -1) * col_stride<DIM>(J, d);
            c[d].lam = (float)d;   // remembers the axis through the sort
        }
    }
    sort_cross<R, DIM>(c);
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const bool ok = k < tot;
        const int a = (int)c[k].lam;
        R la = a == 0 ? lam64[0] : (a == 1 ? lam64[1] : lam64[2]);
        R lc = la > lp ? la : lp;
        lc = lc < le ? lc : le;
        close(ok, wk.cur, (k == 0 ? wk.pend : 0.f) + (float)((lc - lp) * r.Dn));
        wk.cur += ok ? c[k].dcol : 0;
        lp = ok ? lc : lp;
    }
    wk.pend = (tot == 0 ? wk.pend : 0.f) + (float)((le - lp) * r.Dn);
}

// Chord between two spline samples given by voxel index and in-voxel position (voxel
// units, R), at most one crossing per axis.  The displacement and the distance to the
// face are formed in R (no cancellation for a chord nearly parallel to a face), their
// ratio -- the crossing parameter -- and the piece lengths in FP32.
template <typename R, int DIM, class F>
__device__ __forceinline__ void chord_frac(const JobDev &J, const int Ip[3], const R fp[3], const int Ie[3],
                                           const R fe[3], Walker<R> &wk, F &&close) {
    float lam[3], dn2 = 0.f;
    int32_t dcol[3];
    int tot = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lam[d] = 2.f;
        dcol[d] = 0;
        if (d < DIM) {
            const int di = Ie[d] - Ip[d];
            const R df = (di > 0 ? R(1) : (di < 0 ? R(-1) : R(0))) + (fe[d] - fp[d]);   // voxel units
            const float dff = (float)df;
            const float dm = dff * (float)J.h[d];                   // mm
            dn2 = fmaf(dm, dm, dn2);
            const bool up = di > 0;
            tot += di != 0 ? 1 : 0;
            const float dist = (float)(up ? R(1) - fp[d] : fp[d]);
            lam[d] = di != 0 ? dist * __builtin_amdgcn_rcpf(fabsf(dff)) : 2.f;
            dcol[d] = (up ? 1 : -1) * col_stride<DIM>(J, d);
        }
    }
    const float len = __builtin_amdgcn_sqrtf(dn2);
    // order the (at most DIM) crossings; ties keep the lower axis
#define PCT_CSWAP(a, b)                                                  \
    if (lam[b] < lam[a]) {                                               \
        const float tl = lam[a]; lam[a] = lam[b]; lam[b] = tl;           \
        const int32_t tc = dcol[a]; dcol[a] = dcol[b]; dcol[b] = tc;     \
    }
    PCT_CSWAP(0, 1)
    if (DIM == 3) {
        PCT_CSWAP(1, 2)
        PCT_CSWAP(0, 1)
    }
#undef PCT_CSWAP
    float lp = 0.f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
        const bool go = k < tot;
        float lc = lam[k] > lp ? lam[k] : lp;
        lc = lc < 1.f ? lc : 1.f;
        close(go, wk.cur, (k == 0 ? wk.pend : 0.f) + (lc - lp) * len);
        wk.cur += go ? dcol[k] : 0;
        lp = go ? lc : lp;
    }
    wk.pend = (tot == 0 ? wk.pend : 0.f) + (1.f - lp) * len;
}

// Voxel index and in-voxel position (voxel units) of a spline sample.
template <typename R, int DIM>
__device__ __forceinline__ void sample_vox(const JobDev &J, const R p[3], int I[3], R fr[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        I[d] = 0;
        fr[d] = R(0);
        if (d < DIM) {
            const R f = (p[d] - R(J.o[d])) * R(J.invh[d]);
            int v = (int)r_floor<R>(f);
            v = v < 0 ? 0 : (v > J.n[d] - 1 ? J.n[d] - 1 : v);
            I[d] = v;
            fr[d] = f - R(v);
        }
    }
}

// ------------------------------------------------------------------ uniform values
__device__ __forceinline__ double uni(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float uni(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(uint32_t, v)));
}
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <typename R>
__device__ __forceinline__ void uni_ray(RayW<R> &r) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        r.A[d] = uni(r.A[d]);
        r.D[d] = uni(r.D[d]);
        r.invD[d] = uni(r.invD[d]);
        r.is[d] = uni(r.is[d]);
        r.ie[d] = uni(r.ie[d]);
    }
    r.lo = uni(r.lo);
    r.hi = uni(r.hi);
    r.Dn = uni(r.Dn);
    r.dom = uni(r.dom);
    r.sdom = uni(r.sdom);
    r.ncell = uni(r.ncell);
    r.a_dom = uni(r.a_dom);
    r.inv_dom = uni(r.inv_dom);
    r.o_dom = uni(r.o_dom);
    r.h_dom = uni(r.h_dom);
    r.is_dom = uni(r.is_dom);
}

// State carried along a row from block to block and phase to phase.
struct RowCarry {
    int64_t C;         // crossings so far (= index of the open entry)
    float O;           // length accumulated in the open entry
    int32_t open_col;  // its voxel
    bool any;          // at least one item walked
};

// Close the block: the entry open at each lane's start began in an earlier lane (or
// block); its length is the sum of the tail of the last lane with a crossing and the
// whole lengths of the lanes without one (segmented scan), plus this lane's head.
template <typename TW, typename R>
__device__ __forceinline__ void stitch(RowOut<TW> &out, RowCarry &rc, const Walker<R> &wk, int c, int P, int ctot,
                                       int32_t col_start, int lane, int last_lane) {
    const bool f = c > 0;
    int fs = f ? 1 : 0;
    float vs = wk.pend;
    wave_seg_scan(vs, fs);
    const float Oend = fs ? vs : rc.O + vs;   // open length after this lane
    float Oin = __shfl_up(Oend, 1u, WAVE);    // ... before it
    if (lane == 0) Oin = rc.O;
    if (f) out.put((int32_t)rc.C + P, col_start, Oin + wk.head);
    out.fold();
    rc.O = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, Oend), last_lane));
    rc.open_col = __builtin_amdgcn_readlane(wk.cur, last_lane);
    rc.C += ctot;
    rc.any = true;
}

// Cells of one straight ray (uniform RayW), ceil(ncell / 64) consecutive cells per lane:
// a whole ray is one block.  The second pass recomputes the cells (cheap).
template <typename R, int DIM, typename TW>
__device__ __forceinline__ void walk_cells(const JobDev &J, const RayW<R> &r, RowOut<TW> &out, RowCarry &rc,
                                           int lane) {
    const int n = r.ncell;
    if (n == 0) return;
    const int Kr = (n + WAVE - 1) / WAVE;
    const int first = lane * Kr;
    const int lastc = (first + Kr < n) ? first + Kr : n;   // this lane's cells [first, lastc)
    int Is[3] = {0, 0, 0};
    R ls = R(0);
    if (first < n) {
        ls = ray_lam<R>(J, r, first);
        ray_index<R, DIM>(J, r, first, ls, Is);
    }
    // the voxel indices at the cell boundaries are monotone along a ray (clamped that
    // way), so the crossings of the lane's cells are the index differences of its ends
    int c = 0;
    if (first < n) {
        int Ie[3];
        const R le = ray_lam<R>(J, r, lastc);
        ray_index<R, DIM>(J, r, lastc, le, Ie);
#pragma unroll
        for (int d = 0; d < DIM; ++d) c += abs(Ie[d] - Is[d]);
    }
    int ctot;
    const int P = wave_excl_scan(c, lane, ctot);
    const int32_t col_start = col_of<DIM>(J, Is);
    Walker<R> wk;
    wk.head = 0.f;
    wk.pend = 0.f;
    wk.done = 0;
    wk.cur = col_start;
    const int32_t rel0 = (int32_t)rc.C + P;
    auto close = [&](bool ok, int32_t col, float len) {
        if (ok) {
            if (wk.done == 0) wk.head = len;
            else out.put(rel0 + wk.done, col, len);
            ++wk.done;
        }
    };
    {
        int Ip[3] = {Is[0], Is[1], Is[2]};
        R lp = ls;
        for (int m = first; m < lastc; ++m) {
            int Ie[3];
            const R le = ray_lam<R>(J, r, m + 1);
            ray_index<R, DIM>(J, r, m + 1, le, Ie);
            bool one = true;
#pragma unroll
            for (int d = 0; d < DIM; ++d) one = one && abs(Ie[d] - Ip[d]) <= 1;
            if (one) cell_fast<R, DIM>(J, r, Ip, lp, Ie, le, wk, close);
            else cell_pieces<R, DIM>(J, r, Ip, lp, Ie, le, wk, close);
#pragma unroll
            for (int d = 0; d < 3; ++d) Ip[d] = Ie[d];
            lp = le;
        }
    }
    stitch(out, rc, wk, c, P, ctot, col_start, lane, (n - 1) / Kr);
}

// True when every coordinate of the spline is strictly monotone over [s0, s1], with a
// rate that moves each chord by far more than the rounding of a sample: then the voxel
// indices of the computed samples are monotone too, and the crossings between samples
// j0 and j1 add up to the index differences of the two.  x'(s) = c1 + 2 c2 s + 3 c3 s^2.
template <typename R, int DIM>
__device__ __forceinline__ bool spline_monotone(const RowW<R> &w, R s0, R s1) {
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R a = w.c1[d], b = R(2) * w.c2[d], c3 = R(3) * w.c3[d];
        const R g0 = r_fma<R>(r_fma<R>(c3, s0, b), s0, a);
        const R g1 = r_fma<R>(r_fma<R>(c3, s1, b), s1, a);
        R gmin = (g0 < R(0) ? -g0 : g0);
        const R ag1 = (g1 < R(0) ? -g1 : g1);
        gmin = ag1 < gmin ? ag1 : gmin;
        bool same = (g0 > R(0)) == (g1 > R(0));
        // the vertex of the derivative parabola
        if (c3 != R(0)) {
            const R sv = -b / (R(2) * c3);
            if (sv > s0 && sv < s1) {
                const R gv = r_fma<R>(r_fma<R>(c3, sv, b), sv, a);
                same = same && ((gv > R(0)) == (g0 > R(0)));
                const R agv = gv < R(0) ? -gv : gv;
                gmin = agv < gmin ? agv : gmin;
            }
        }
        ok = ok && same && (gmin * w.invN > R(sizeof(R) == 8 ? 1e-9 : 1e-2));
    }
    return ok;
}

// Chords of the spline (N of them, samples 0..N): ceil(N / 64) consecutive chords per
// lane, so a whole spline is one block.  The first pass reads the crossing count off the
// lane's first and last samples when the spline is monotone there, else sample by sample;
// the second pass walks the chords.
template <typename R, int DIM, typename TW>
__device__ __forceinline__ void walk_chords(const JobDev &J, const RowW<R> &w, RowOut<TW> &out, RowCarry &rc,
                                            int lane) {
    const int n = w.N;
    const int K = (n + WAVE - 1) / WAVE;
    const int first = lane * K;
    const int lastc = (first + K < n) ? first + K : n;
    int Is[3] = {0, 0, 0};
    R fs[3] = {R(0), R(0), R(0)};
    int c = 0;
    if (first < n) {
        R Ps[3], Pe[3];
        spline_at<R, DIM>(w, first, Ps);
        sample_vox<R, DIM>(J, Ps, Is, fs);
        const R s0 = R(first) * w.invN, s1 = R(lastc) * w.invN;
        if (spline_monotone<R, DIM>(w, s0, s1)) {
            int Ie[3];
            R fe[3];
            spline_at<R, DIM>(w, lastc, Pe);
            sample_vox<R, DIM>(J, Pe, Ie, fe);
#pragma unroll
            for (int d = 0; d < DIM; ++d) c += abs(Ie[d] - Is[d]);
        } else {
            int Ip[3] = {Is[0], Is[1], Is[2]};
            for (int j = first + 1; j <= lastc; ++j) {
                int Ie[3];
                R fe[3];
                spline_at<R, DIM>(w, j, Pe);
                sample_vox<R, DIM>(J, Pe, Ie, fe);
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    c += abs(Ie[d] - Ip[d]);
                    Ip[d] = Ie[d];
                }
            }
        }
    }
    int ctot;
    const int P = wave_excl_scan(c, lane, ctot);
    const int32_t col_start = col_of<DIM>(J, Is);
    Walker<R> wk;
    wk.head = 0.f;
    wk.pend = 0.f;
    wk.done = 0;
    wk.cur = col_start;
    const int32_t rel0 = (int32_t)rc.C + P;
    auto close = [&](bool ok, int32_t col, float len) {
        if (ok) {
            if (wk.done == 0) wk.head = len;
            else out.put(rel0 + wk.done, col, len);
            ++wk.done;
        }
    };
    {
        int Ip[3] = {Is[0], Is[1], Is[2]};
        R fp[3] = {fs[0], fs[1], fs[2]};
        for (int j = first; j < lastc; ++j) {
            R Pe[3];
            int Ie[3];
            R fe[3];
            spline_at<R, DIM>(w, j + 1, Pe);
            sample_vox<R, DIM>(J, Pe, Ie, fe);
            bool one = true;
#pragma unroll
            for (int d = 0; d < DIM; ++d) one = one && abs(Ie[d] - Ip[d]) <= 1;
            if (one) {
                chord_frac<R, DIM>(J, Ip, fp, Ie, fe, wk, close);
            } else {
                R Pa[3];
                spline_at<R, DIM>(w, j, Pa);
                chord_pieces<R, DIM>(J, Ip, Pa, Ie, Pe, wk, close);
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                Ip[d] = Ie[d];
                fp[d] = fe[d];
            }
        }
    }
    stitch(out, rc, wk, c, P, ctot, col_start, lane, (n - 1) / K);
}

// Walk one row with the whole wave, in three phases that hold only their own data:
// the first ray, the spline chords, the last ray.  n_entries = entries produced.
template <typename R, int DIM, int KR, int KC, typename TW>
__device__ __forceinline__ void wave_row(const JobDev &J, const RowW<R> &w, int kind, RowOut<TW> &out, int lane,
                                         int64_t &n_entries) {
    RowCarry rc;
    rc.C = 0;
    rc.O = 0.f;
    rc.open_col = -1;
    rc.any = false;
    walk_cells<R, DIM, TW>(J, w.ray[0], out, rc, lane);
    if (kind == 2) {
        walk_chords<R, DIM, TW>(J, w, out, rc, lane);
        walk_cells<R, DIM, TW>(J, w.ray[1], out, rc, lane);
    }
    if (rc.any) {
        if (lane == 0) out.put((int32_t)rc.C, rc.open_col, rc.O);
        out.fold();
        n_entries = rc.C + 1;
    } else {
        n_entries = 0;
    }
}

// ------------------------------------------------------------------ row setup (one lane)
template <typename R, int DIM>
__device__ __forceinline__ bool hull_inside(const JobDev &J, const R p[3]) {
    const R m = sizeof(R) == 8 ? R(1e-9) : R(1e-3);
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) ok = ok && (p[d] >= R(J.o[d]) + m) && (p[d] <= R(J.top[d]) - m);
    return ok;
}

template <typename R, int DIM>
__device__ __forceinline__ void setup_row(const JobDev &J, int64_t g, RowW<R> &w) {
    PathGeom<R> p;
    if (J.path == 1) make_path<R, DIM, true>(J, g, p);
    else make_path<R, DIM, false>(J, g, p);
    const R ninf = -r_inf<R>(), pinf = r_inf<R>();
    w.N = 0;
    if (!p.curved) {
        R lo = ninf, hi = pinf;
        const bool hit = clip_box<R, DIM>(J, p.Q, p.u, lo, hi);
        w.kind = hit ? 1 : 0;
        if (!hit) { lo = R(1); hi = R(0); }
        ray_prepare<R, DIM>(J, p.Q, p.u, lo, hi, w.ray[0]);
    } else {
        // the spline lies in the convex hull of its Bezier control points
        R b1[3], b2[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            b1[d] = p.P0[d] + p.L * p.d0[d] / R(3);
            b2[d] = p.P1[d] - p.L * p.d1[d] / R(3);
        }
        const bool in = hull_inside<R, DIM>(J, p.P0) && hull_inside<R, DIM>(J, p.P1) &&
                        hull_inside<R, DIM>(J, b1) && hull_inside<R, DIM>(J, b2);
        w.kind = in ? 2 : 3;
        R lo = ninf, hi = R(0);
        if (!clip_box<R, DIM>(J, p.P0, p.d0, lo, hi)) { lo = R(1); hi = R(0); }
        ray_prepare<R, DIM>(J, p.P0, p.d0, lo, hi, w.ray[0]);
        lo = R(0);
        hi = pinf;
        if (!clip_box<R, DIM>(J, p.P1, p.d1, lo, hi)) { lo = R(1); hi = R(0); }
        ray_prepare<R, DIM>(J, p.P1, p.d1, lo, hi, w.ray[1]);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            w.c1[d] = p.c1[d];
            w.c2[d] = p.c2[d];
            w.c3[d] = p.c3[d];
        }
        w.N = p.N;
        w.invN = p.invN;
    }
    w.bfac = 1.0;
    if (J.noise > 0.0) {
        R z1, z2;
        normal_pair<R>(J.seed, 4, (uint64_t)g, z1, z2);
        w.bfac = (double)(R(1) + R(J.noise) * z1);
    }
}

// Wave part of the emit kernel for rows [r0, r0 + 64) of job J (one wavefront).
// Number of CSR entries of a row described by w (one lane): 1 + the face crossings of
// its items, exactly as wave_row produces them; the per-lane walk for kind 3.
template <typename R, int DIM>
__device__ __forceinline__ int64_t count_row(const JobDev &J, const RowW<R> &w, int64_t g) {
    if (w.kind == 0) return 0;
    if (w.kind == 3) {
        CountSink s;
        trace_row<R, DIM, true>(J, g, s);
        return s.n;
    }
    int64_t c = 0;
    bool any = false;
    if (w.ray[0].ncell > 0) {
#pragma unroll
        for (int d = 0; d < DIM; ++d) c += abs(w.ray[0].ie[d] - w.ray[0].is[d]);
        any = true;
    }
    if (w.kind == 2) {
        R A[3];
        spline_at<R, DIM>(w, 0, A);
        int Ia[3];
        spline_index<R, DIM>(J, A, Ia);
        for (int j = 1; j <= w.N; ++j) {
            R B[3];
            spline_at<R, DIM>(w, j, B);
            int Ib[3];
            spline_index<R, DIM>(J, B, Ib);
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                c += abs(Ib[d] - Ia[d]);
                Ia[d] = Ib[d];
            }
        }
        any = true;
        if (w.ray[1].ncell > 0) {
#pragma unroll
            for (int d = 0; d < DIM; ++d) c += abs(w.ray[1].ie[d] - w.ray[1].is[d]);
        }
    }
    return any ? c + 1 : 0;
}

// Emit pass over rows [r0, r0 + 64) of job J by one wavefront; w points at the job's
// row descriptions.
template <typename R, int DIM, int KR, int KC, bool STORE>
__device__ __forceinline__ void emit_rows_wave(const JobDev &J, const RowW<R> *__restrict__ rows, int64_t r0,
                                               int lane, int32_t *status) {
    using TW = typename std::conditional<std::is_same<R, double>::value, double, float>::type;
    const int64_t rend = (r0 + WAVE < J.row_count) ? r0 + WAVE : J.row_count;
    for (int64_t r = r0; r < rend; ++r) {
        const RowW<R> &w = rows[r];
        const int kind = w.kind;
        if (kind == 3) continue;   // walked by the per-lane kernel
        RowOut<TW> out;
        out.x = J.x;
        out.wepl = 0.f;
        out.wacc = TW(0);
        out.half = (J.val_dtype == PCT_F16);
        out.want_b = (J.b != nullptr);
        out.store = STORE;
        out.len = 0;
        int64_t pos = 0;
        if (STORE) {
            pos = J.row_ptr[r];
            const int64_t end = J.row_ptr[r + 1];
            if (pos < 0 || end < pos || end > J.cap) {
                if (lane == 0) set_status_dev(status, PCT_ECAPACITY);
                out.store = false;
                pos = 0;
            } else {
                out.len = (int32_t)(end - pos);
            }
        }
        out.cols = J.cols + pos;
        out.vh = (__half *)J.vals + pos;
        out.vf = (float *)J.vals + pos;
        int64_t ne = 0;
        if (kind != 0) wave_row<R, DIM, KR, KC, TW>(J, w, kind, out, lane, ne);
        if (out.store && ne != out.len && lane == 0) set_status_dev(status, PCT_EINTERNAL);
        if (out.want_b) {
            const TW bs = (TW)wave_sum((double)out.wacc);
            if (lane == 0) J.b[r] = (float)(bs * (TW)w.bfac);
        }
    }
}

// Rows whose spline may leave the box (kind 3): one lane per row, general walk.
template <typename R, int DIM, bool STORE>
__device__ __forceinline__ void emit_row_lane(const JobDev &J, const RowW<R> &w, int64_t r, int32_t *status) {
    using TW = typename std::conditional<std::is_same<R, double>::value, double, float>::type;
    EmitSink<R, TW> s;
    s.cols = J.cols;
    s.vals = J.vals;
    s.x = J.x;
    s.half = (J.val_dtype == PCT_F16);
    s.want_b = (J.b != nullptr);
    s.store = STORE;
    s.pos = 0;
    s.end = 0;
    if (STORE) {
        s.pos = J.row_ptr[r];
        s.end = J.row_ptr[r + 1];
        if (s.pos < 0 || s.end < s.pos || s.end > J.cap) {
            s.store = false;
            set_status_dev(status, PCT_ECAPACITY);
        }
    }
    trace_row<R, DIM, true>(J, J.row_begin + r, s);
    s.flush();
    if (s.store && s.pos != s.end) set_status_dev(status, PCT_EINTERNAL);
    if (s.want_b) J.b[r] = (float)(s.wepl * (TW)w.bfac);
}

}  // namespace pct

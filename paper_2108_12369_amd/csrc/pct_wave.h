// pct_wave.h -- wave-cooperative emit of CSR rows (gfx950, wave64).
//
// A row's path is a sequence of "items", straight steps between two points whose voxels
// are known:
//   - a ray inside the grid box (the whole straight path, or the part before the entry
//     point or after the exit point of a curved path) is cut at the faces of its
//     dominant axis, the axis crossed most often per unit length, so that an item
//     crosses every axis at most once;
//   - the spline is cut at its samples, one item per chord.
// Positions are kept in voxel units, F = (p - o) / h, and the end of item m is a
// polynomial in m (linear on a ray, cubic on the spline), so any lane can evaluate any
// item end directly.
//
// One wavefront walks one row.  Its pieces (ray, spline, ray) get consecutive groups
// of lanes, each lane K consecutive items of its piece, K the same for the whole row.
// Pass 1: each lane finds the voxels at its first and last item end and the number of
// face crossings between them: the index difference where the indices are monotone
// over the lane's items (always on a ray; on the spline away from the turning points
// of a coordinate, which the count pass records), else by walking the samples.  A wave
// prefix sum of those counts places every lane's entries in the row.
// Pass 2: each lane walks its items, orders the crossings inside each item and writes
// the entries that close inside the lane.  The entry open at a lane's start began in
// an earlier lane: its length comes from a segmented scan over the lanes, and the lane
// that closes it writes it.  The stores of a row form one contiguous range written by
// the whole wave.
// A straight row in the mixed form (FP64 geometry) has no items in pass 2: each lane
// takes its crossings directly in the order of the ray parameter, and every entry's
// length is measured from the row's previous crossing, so there is no stitch
// (wave_ray_row).
//
// The count pass (one lane per row) writes each row's description and counts its
// entries, 1 + (face crossings), with the same item ends and the same index rule as
// the walk, so the two passes agree exactly.  Rows whose spline may leave the grid box
// are walked by the per-lane code (trace_row) instead.
#pragma once

#include "pct_device.h"

namespace pct {

constexpr int WAVE = 64;

// A ray inside the box, A + l D for l in [lo, hi], cut into M items at the faces of its
// dominant axis.  Item ends 0 < m < M lie on those faces: F(m) = c0 + c1 m.  The ends
// of the ray are the same line at the parameters tS (in [0, 1]) and tE (in [M-1, M]):
// item end m is F(min(max(m, tS), tE)).  On the dominant axis F(tS) is the clipped start
// point exactly; elsewhere the ends agree with the clipped points to rounding.
template <typename R>
struct RayP {
    R c0[3], c1[3];
    R tS, tE;
    int32_t M;              // items; 0 when the ray misses the box
    int32_t lo[3], hi[3];   // voxel index range between the end voxels, per axis
};

// The spline between entry and exit: N items, one per chord.  Sample m (0 <= m <= N) is
// F(m) = ((c3 m + c2) m + c1) m + c0: c0 is the entry point, F(N) the exit point to
// rounding.  win: per axis up to two sample ranges [a, b] (a < b; unused: -1, -1)
// outside of which the computed samples are strictly monotone in that coordinate.
template <typename R>
struct SplP {
    R c0[3], c1[3], c2[3], c3[3];
    int32_t N;
    int32_t win[3][4];
};

// Per-row path description, written by the count pass into the workspace.
template <typename R>
struct RowV {
    int32_t kind;           // 0: no entry, 1: one ray, 2: ray + spline + ray, 3: per-lane walk
    int32_t fast;           // every item crosses each axis at most once
    double bfac;            // WEPL noise factor 1 + r z
    RayP<R> ray[2];         // ray[0]: the straight path, or the ray into the entry point
    SplP<R> spl;
};

// Storage of the descriptions.  Each job has RV_TILE * rv_bytes bytes per count tile.
// Inside it, rows are grouped by 2^S: 16-byte chunk c of row i of a group sits at byte
// (c * 2^S + i) * 16 of the group's block.  S = 8, for 2D and 3D grids alike:
// chunk-transposed over a whole tile, so that the count pass (one lane per row) writes
// every chunk of 64 consecutive rows with one contiguous 1 KiB store.  (With each row
// contiguous, S = 0, the emit reads a row from 4 cache lines instead of 23, but every
// store of the count pass touches 64 lines: the 3D count took 3.7 ms on the 64-job
// batch instead of 2.2, the 3D emit 19.2 ms instead of 19.4.)
// A field never straddles a chunk (all are 4 or 8 bytes at their natural alignment).
constexpr int RV_TILE = 256;
template <typename R>
constexpr size_t rv_bytes() { return (sizeof(RowV<R>) + 15) & ~size_t(15); }
template <int DIM>
constexpr int rv_shift() { return 8; }

template <typename R, int S>
struct RowRef {
    char *tb;    // the row's group block
    int i;       // row in the group
    template <class T>
    __device__ __forceinline__ T &at(size_t off) const {
        return *reinterpret_cast<T *>(tb + ((((off >> 4) << S) + (size_t)i) << 4) + (off & 15));
    }
};
template <typename R, int DIM>
using RowRefD = RowRef<R, rv_shift<DIM>()>;

// A row description copied into the wave's LDS: chunk c at byte 16 c.
struct LdsRow {
    char *p;
    template <class T>
    __device__ __forceinline__ T &at(size_t off) const {
        return *reinterpret_cast<T *>(p + off);
    }
};

// The description of row r of job J.
template <typename R, int DIM>
__device__ __forceinline__ RowRefD<R, DIM> row_ref(char *rowbuf, const JobDev &J, int64_t r) {
    constexpr int S = rv_shift<DIM>();
    char *jb = rowbuf + J.tile_base * (int64_t)(RV_TILE * rv_bytes<R>());
    const int64_t grp = r >> S;
    return RowRefD<R, DIM>{jb + grp * (int64_t)(rv_bytes<R>() << S), (int)(r & ((1 << S) - 1))};
}

#define RV(w, member) \
    (w).template at<typename std::remove_reference<decltype(((RowV<R> *)nullptr)->member)>::type>( \
        __builtin_offsetof(RowV<R>, member))

// Lane i's value of v, as a wave-uniform value.
__device__ __forceinline__ int64_t readlane_i64(int64_t v, int i) {
    const uint64_t u = (uint64_t)v;
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, i);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), i);
    return (int64_t)(lo | (hi << 32));
}

// A field of the current row's description, read from the wave's LDS copy (one read
// for the wave, no trip to memory) and made wave-uniform.
__device__ __forceinline__ int32_t uniform_i32(const LdsRow &wl, size_t off) {
    return __builtin_amdgcn_readfirstlane(wl.template at<int32_t>(off));
}
__device__ __forceinline__ double uniform_f64(const LdsRow &wl, size_t off) {
    const uint2 v = wl.template at<uint2>(off);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)v.x);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)v.y);
    return __builtin_bit_cast(double, lo | (hi << 32));
}
#define RL_I32(wl, member) uniform_i32((wl), __builtin_offsetof(RowV<R>, member))
#define RL_F64(wl, member) uniform_f64((wl), __builtin_offsetof(RowV<R>, member))

template <typename R> __device__ __forceinline__ R r_fmax(R a, R b) {
    if constexpr (std::is_same<R, float>::value) return fmaxf(a, b); else return fmax(a, b);
}
template <typename R> __device__ __forceinline__ R r_fmin(R a, R b) {
    if constexpr (std::is_same<R, float>::value) return fminf(a, b); else return fmin(a, b);
}

// One piece of a row as a lane walks it: item end m is the polynomial at
// t = min(max(m, tS), tE), its voxel index clamped into [lo, hi] per axis.
template <typename R>
struct LaneP {
    R c0[3], c1[3], c2[3], c3[3];
    R tS, tE;               // parameters of the piece's ends
    int32_t lo[3], hi[3];   // voxel index range of the piece
    int32_t M;
};

// ---------------------------------------------------------------- row description
// The part of A + l D (l in [lo, hi], already clipped to the box) as a ray piece.
// Returns false when a minor axis moves (almost) as fast as the dominant one: an item
// could then cross it twice through rounding.
template <typename R, int DIM, int WHICH>
__device__ __forceinline__ bool make_ray(const JobDev &J, const R A[3], const R D[3], R lo, R hi, bool hit,
                                         RowRefD<R, DIM> w, LaneP<R> &lp) {
    R Av[3] = {R(0), R(0), R(0)}, Dv[3] = {R(0), R(0), R(0)};
    R Fs[3] = {R(0), R(0), R(0)}, Fe[3] = {R(0), R(0), R(0)};
    int is[3] = {0, 0, 0}, ie[3] = {0, 0, 0};
    int dom = 0;
    R best = R(-1);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R ih = R(J.invh[d]);
        Av[d] = (A[d] - R(J.o[d])) * ih;
        Dv[d] = D[d] * ih;
        const R P = A[d] + lo * D[d];
        const R E = A[d] + hi * D[d];
        Fs[d] = (P - R(J.o[d])) * ih;
        Fe[d] = (E - R(J.o[d])) * ih;
        is[d] = vox_index<R>(P, J.o[d], J.invh[d], J.n[d]);
        ie[d] = vox_index<R>(E, J.o[d], J.invh[d], J.n[d]);
        const R rate = Dv[d] < R(0) ? -Dv[d] : Dv[d];
        if (rate > best) {
            best = rate;
            dom = d;
        }
    }
    int isd = 0, ied = 0;
    R avd = R(0), dvd = R(1), fsd = R(0), fed = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d)
        if (d == dom) {
            isd = is[d];
            ied = ie[d];
            avd = Av[d];
            dvd = Dv[d];
            fsd = Fs[d];
            fed = Fe[d];
        }
    // the direction along the dominant axis (a ray inside one voxel of that axis moves
    // one way too: its end parameters keep tS <= tE)
    const int sdom = dvd >= R(0) ? 1 : -1;
    // face of item end m: isd + m (upwards) or isd + 1 - m (downwards)
    const R c0d = R(sdom > 0 ? isd : isd + 1), c1d = R(sdom);
    bool one = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R c0 = R(0), c1 = R(0);
        int lo_ = 0, hi_ = 0;
        if (d < DIM) {
            lo_ = is[d] < ie[d] ? is[d] : ie[d];
            hi_ = is[d] < ie[d] ? ie[d] : is[d];
            if (d == dom) {
                c0 = c0d;
                c1 = c1d;
            } else {
                const R rd = Dv[d] / dvd;
                c0 = r_fma<R>(c0d - avd, rd, Av[d]);
                c1 = c1d * rd;
                if (!((rd < R(0) ? -rd : rd) < R(0.999))) one = false;
            }
        }
        RV(w, ray[WHICH].c0[d]) = c0;
        RV(w, ray[WHICH].c1[d]) = c1;
        RV(w, ray[WHICH].lo[d]) = lo_;
        RV(w, ray[WHICH].hi[d]) = hi_;
        // the piece as the emit reads it back (lane_ray: the range kept inside the grid)
        const int top = J.n[d] - 1;
        const int clo = lo_ < 0 ? 0 : (lo_ > top ? top : lo_);
        lp.c0[d] = c0;
        lp.c1[d] = c1;
        lp.c2[d] = R(0);
        lp.c3[d] = R(0);
        lp.lo[d] = clo;
        lp.hi[d] = hi_ < clo ? clo : (hi_ > top ? top : hi_);
    }
    const int32_t M = hit ? abs(ied - isd) + 1 : 0;
    // end parameters on the dominant axis (c1 = +-1): F(t) = c0 + c1 t
    const R tS = hit ? (fsd - c0d) * c1d : R(0), tE = hit ? (fed - c0d) * c1d : R(0);
    RV(w, ray[WHICH].M) = M;
    RV(w, ray[WHICH].tS) = tS;
    RV(w, ray[WHICH].tE) = tE;
    lp.M = M;
    lp.tS = tS;
    lp.tE = tE;
    return one;
}

// Whether |F'(m)| = |c1 + 2 c2 m + 3 c3 m^2| stays above thr with one sign over [s0, s1]
// (true for an empty range): the smallest |F'| is at an end or at the vertex of F'.
template <typename R>
__device__ __forceinline__ bool rate_ok(R qa, R qb, R qc, R mv, int s0i, int s1i, R thr) {
    if (s1i <= s0i) return true;
    const R s0 = R(s0i), s1 = R(s1i);
    const R g0 = r_fma<R>(r_fma<R>(qa, s0, qb), s0, qc);
    const R g1 = r_fma<R>(r_fma<R>(qa, s1, qb), s1, qc);
    bool same = (g0 > R(0)) == (g1 > R(0));
    R gmin = r_fmin<R>(g0 < R(0) ? -g0 : g0, g1 < R(0) ? -g1 : g1);
    if (mv > s0 && mv < s1) {
        const R gv = r_fma<R>(r_fma<R>(qa, mv, qb), mv, qc);
        same = same && ((gv > R(0)) == (g0 > R(0)));
        gmin = r_fmin<R>(gmin, gv < R(0) ? -gv : gv);
    }
    return same && gmin > thr;
}

// Sample ranges of one spline coordinate F(m) where consecutive computed samples may
// fail to be strictly monotone: around the roots of F'(m) = c1 + 2 c2 m + 3 c3 m^2 in
// the sampled range, and any stretch between them where |F'| (the step per chord)
// drops below `thr` -- far above the rounding of a sample, so that outside the ranges
// the computed samples keep the order of the exact ones.  Up to two ranges [a, b]
// (a < b; unused: -1, -1), merged conservatively.
template <typename R>
__device__ __forceinline__ void spline_windows(R c1, R c2, R c3, int N, R thr, int32_t win[4]) {
    const R qa = R(3) * c3, qb = R(2) * c2, qc = c1;
    R rt0 = R(0), rt1 = R(0);
    int nr = 0;
    if (qa != R(0)) {
        const R disc = qb * qb - R(4) * qa * qc;
        if (disc >= R(0)) {
            const R sq = r_sqrt<R>(disc);
            const R t = (qb >= R(0)) ? -(qb + sq) : (sq - qb);
            const R r1 = t / (R(2) * qa);
            const R r2 = (t != R(0)) ? (R(2) * qc) / t : r1;
            rt0 = r1 < r2 ? r1 : r2;
            rt1 = r1 < r2 ? r2 : r1;
            nr = 2;
        }
    } else if (qb != R(0)) {
        rt0 = -qc / qb;
        nr = 1;
    }
    // windows of two samples on either side of each root in (-1, N + 1)
    bool v0 = false, v1 = false;
    int wa0 = 0, wb0 = 0, wa1 = 0, wb1 = 0;
    if (nr >= 1 && rt0 > R(-1) && rt0 < R(N + 1)) {
        v0 = true;
        wa0 = max((int)r_floor<R>(rt0) - 1, 0);
        wb0 = min((int)r_ceil<R>(rt0) + 1, N);
    }
    if (nr >= 2 && rt1 > R(-1) && rt1 < R(N + 1)) {
        v1 = true;
        wa1 = max((int)r_floor<R>(rt1) - 1, 0);
        wb1 = min((int)r_ceil<R>(rt1) + 1, N);
    }
    if (!v0 && v1) {
        v0 = true;
        wa0 = wa1;
        wb0 = wb1;
        v1 = false;
    }
    if (v0 && v1 && wa1 <= wb0) {   // overlapping windows
        wb0 = max(wb0, wb1);
        v1 = false;
    }
    // segments of [0, N] in order: interval, window, interval, window, interval; an
    // interval whose rate is too small becomes unsafe as well
    const R mv = (qa != R(0)) ? -qb / (R(2) * qa) : R(-1);
    const int e0 = v0 ? wa0 : N;
    const int s1 = v0 ? wb0 : N, e1 = v1 ? wa1 : N;
    const int s2 = v1 ? wb1 : N;
    int sa[5] = {0, wa0, s1, wa1, s2};
    int sb[5] = {e0, wb0, e1, wb1, N};
    bool bad[5] = {!rate_ok<R>(qa, qb, qc, mv, 0, e0, thr), v0, v0 && !rate_ok<R>(qa, qb, qc, mv, s1, e1, thr), v1,
                   v1 && !rate_ok<R>(qa, qb, qc, mv, s2, N, thr)};
    // merge adjacent unsafe segments; at most two ranges remain
    int a0 = -1, b0 = -1, a1 = -1, b1 = -1, nw = 0;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        if (!bad[k] || sb[k] <= sa[k]) continue;
        if (nw == 1 && b0 >= sa[k]) {
            b0 = max(b0, sb[k]);
        } else if (nw == 2 && b1 >= sa[k]) {
            b1 = max(b1, sb[k]);
        } else if (nw == 0) {
            a0 = sa[k];
            b0 = sb[k];
            nw = 1;
        } else if (nw == 1) {
            a1 = sa[k];
            b1 = sb[k];
            nw = 2;
        } else {
            b1 = sb[k];   // a third range: widen the second one over the gap
        }
    }
    win[0] = a0;
    win[1] = b0;
    win[2] = a1;
    win[3] = b1;
}

// ---------------------------------------------------------------- per-lane piece

// The index range is kept inside the grid whatever the description holds, so that no
// column can leave x.
template <typename R, int DIM, int WHICH, class W>
__device__ __forceinline__ void lane_ray(const JobDev &J, W w, LaneP<R> &p) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p.c0[d] = RV(w, ray[WHICH].c0[d]);
        p.c1[d] = RV(w, ray[WHICH].c1[d]);
        p.c2[d] = R(0);
        p.c3[d] = R(0);
        const int top = J.n[d] - 1;
        const int rlo = RV(w, ray[WHICH].lo[d]), rhi = RV(w, ray[WHICH].hi[d]);
        const int lo = rlo < 0 ? 0 : (rlo > top ? top : rlo);
        const int hi = rhi < lo ? lo : (rhi > top ? top : rhi);
        p.lo[d] = lo;
        p.hi[d] = hi;
    }
    p.tS = RV(w, ray[WHICH].tS);
    p.tE = RV(w, ray[WHICH].tE);
    p.M = RV(w, ray[WHICH].M);
}

template <typename R, int DIM, class W>
__device__ __forceinline__ void lane_spline(const JobDev &J, W w, LaneP<R> &p) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p.c0[d] = RV(w, spl.c0[d]);
        p.c1[d] = RV(w, spl.c1[d]);
        p.c2[d] = RV(w, spl.c2[d]);
        p.c3[d] = RV(w, spl.c3[d]);
        p.lo[d] = 0;
        p.hi[d] = J.n[d] - 1;
    }
    p.M = RV(w, spl.N);
    p.tS = R(0);
    p.tE = R(p.M);
}

// End of item m - 1 (m = 0: the piece's start point).  mf == m.
template <typename R, int DIM>
__device__ __forceinline__ void piece_point(const LaneP<R> &p, int m, R mf, R F[3]) {
    (void)m;
    const R t = r_fmin<R>(r_fmax<R>(mf, p.tS), p.tE);
#pragma unroll
    for (int d = 0; d < 3; ++d)
        F[d] = d < DIM ? r_fma<R>(r_fma<R>(r_fma<R>(p.c3[d], t, p.c2[d]), t, p.c1[d]), t, p.c0[d]) : R(0);
}

// Same, for m >= 1 >= tS (or a piece with tS = tE = 0): the same point as piece_point.
template <typename R, int DIM>
__device__ __forceinline__ void piece_next(const LaneP<R> &p, int m, R mf, R F[3]) {
    (void)m;
    const R t = r_fmin<R>(mf, p.tE);
#pragma unroll
    for (int d = 0; d < 3; ++d)
        F[d] = d < DIM ? r_fma<R>(r_fma<R>(r_fma<R>(p.c3[d], t, p.c2[d]), t, p.c1[d]), t, p.c0[d]) : R(0);
}

// Voxel of a point and its position in that voxel (voxel units).  The index is kept in
// the piece's range: the end voxels of a ray, the grid for the spline.  A ray's end on
// the grid box can round to just outside it; the position is then taken in the voxel
// the index keeps (slightly below 0 or above 1), so that the face distances stay right.
template <typename R, int DIM>
__device__ __forceinline__ void piece_voxel(const LaneP<R> &p, const R F[3], int I[3], R fr[3]) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        I[d] = 0;
        fr[d] = R(0);
        if (d < DIM) {
            // truncation equals the floor for F >= 0, and the range starts at 0 or above,
            // so this is the floor clamped into [lo, hi] (a conversion that saturates
            // keeps any F in the range)
            const int t = (int)F[d];
            I[d] = min(max(t, p.lo[d]), p.hi[d]);
            fr[d] = F[d] - R(I[d]);
        }
    }
}

// Voxel index along axis d of item end m of a piece: the arithmetic of piece_point and
// piece_voxel on that axis alone.
template <typename R>
__device__ __forceinline__ int axis_index(const LaneP<R> &p, int d, R mf) {
    const R t = r_fmin<R>(r_fmax<R>(mf, p.tS), p.tE);
    const R F = r_fma<R>(r_fma<R>(r_fma<R>(p.c3[d], t, p.c2[d]), t, p.c1[d]), t, p.c0[d]);
    return min(max((int)F, p.lo[d]), p.hi[d]);
}

// Crossings of a ray piece: its voxel indices are monotone over the item ends, so per
// axis the difference of the indices at its two ends.
template <typename R, int DIM>
__device__ __forceinline__ int64_t ray_piece_crossings(const LaneP<R> &p) {
    int64_t c = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) c += abs(axis_index<R>(p, d, R(p.M)) - axis_index<R>(p, d, R(0)));
    return c;
}

// Crossings of the spline along axis d: index differences over the monotone stretches,
// sample by sample inside the recorded windows.
template <typename R>
__device__ __forceinline__ int64_t spline_axis_crossings(const LaneP<R> &p, int d, const int32_t win[4]) {
    int64_t c = 0;
    int Iprev = axis_index<R>(p, d, R(0));
    for (int k = 0; k < 2; ++k) {
        const int a = win[2 * k], b = win[2 * k + 1];
        if (a < 0) continue;
        int Ia = axis_index<R>(p, d, R(a));
        c += abs(Ia - Iprev);
        for (int j = a + 1; j <= b; ++j) {
            const int Ij = axis_index<R>(p, d, R(j));
            c += abs(Ij - Ia);
            Ia = Ij;
        }
        Iprev = Ia;
    }
    return c + abs(axis_index<R>(p, d, R(p.M)) - Iprev);
}

// ------------------------------------------------------------------ wave helpers
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

__device__ __forceinline__ int wave_excl_scan(int v, int &total) {
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

// DPP move of a 64-bit value (two 32-bit moves with the same control).
template <int CTRL, int ROWMASK, bool BOUND>
__device__ __forceinline__ double dpp_f64(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, CTRL, ROWMASK, 0xf, BOUND);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), CTRL, ROWMASK, 0xf, BOUND);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the wavefront (the same DPP steps as the integer scan; the total ends in
// lane 63), returned to every lane.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_f64<0x111, 0xf, true>(v);
    v += dpp_f64<0x112, 0xf, true>(v);
    v += dpp_f64<0x114, 0xf, true>(v);
    v += dpp_f64<0x118, 0xf, true>(v);
    v += dpp_f64<0x142, 0xa, false>(v);
    v += dpp_f64<0x143, 0xc, false>(v);
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, WAVE - 1);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), WAVE - 1);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Value of the previous lane (lane 0: 0), DPP wave_shr:1.
__device__ __forceinline__ float lane_prev(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xf, 0xf, false));
}

// Entries a wavefront keeps in LDS per row (8 B each: column, FP32 length).  The slice
// has STAGE_CAP + 1 = 1024 slots (a power of two, so an index is kept inside it by a
// mask) and a row the wave walks has at most STAGE_CAP entries; a block of four waves
// uses 32 KiB, which keeps 5 blocks on a CU.  The last STAGE_DESC slots also hold the
// wave's copy of the current row's description: a row of more than STAGE_ROW_MAX
// entries overwrites it, and the next row's copy is then written after the row's stores.
constexpr int STAGE_CAP = 1023;
constexpr int STAGE_DESC = (int)(rv_bytes<double>() / 8);
constexpr int STAGE_ROW_MAX = STAGE_CAP + 1 - STAGE_DESC;
static_assert(rv_bytes<double>() % 16 == 0 && STAGE_ROW_MAX % 2 == 0, "the copy is 16-byte aligned");

// Output of one row: the row's entries are staged in the wave's LDS slice (at most
// STAGE_CAP; longer rows are walked by the per-lane kernel) and written out afterwards
// in order, 64 consecutive entries per store instruction, into the row's slices of
// cols / vals.  WEPL partial per lane in FP32 over the lane's pieces, folded into TW.
// Pointers into device memory in the global address space: loads and stores become
// global_* instructions, counted by vmcnt only (a generic pointer gives flat_*
// instructions, which every wait for a scalar or LDS access also waits for).
#define PCT_GLOBAL __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ PCT_GLOBAL T *gptr(T *p) { return (PCT_GLOBAL T *)p; }


// Bit offsets of y and z in the packed voxel coordinates of a staged entry (stage_strides).
constexpr int PACK_Y = 10, PACK_Z = 21;

template <typename TW>
struct RowOut {
    PCT_GLOBAL int32_t *cols;
    PCT_GLOBAL uint16_t *vh;   // binary16 bits
    PCT_GLOBAL float *vf;
    PCT_GLOBAL const float *x;
    PCT_GLOBAL const float *xb;   // the bricked copy of x (staged entries hold packed
    bool pack;                    // coordinates); gn: grid sizes, nbx, nby: bricks per
    uint32_t gn[3], nbx, nby;     // grid row and per plane
    uint2 *stage;   // the wave's LDS slice
    uint32_t nvox;  // size of x: every gather index is kept below it
    int32_t len;
    float chord;    // > 0: stored instead of the length (b keeps the length)
    float wepl;
    TW wacc;
    bool store, half, want_b;
    bool bad;       // a lane closed another number of entries than it counted
    // the next row's description, fetched while this row is walked (one 16-byte chunk in
    // each of the first dnc lanes), is waited for before this row's stores and gathers
    // are issued, so that the wait covers nothing newer, and on every path through the
    // row, so that no fetch is pending when the next one reuses its registers.
    uint4 *dbuf;
    uint4 dnext;
    int dnc;

    // wait for the fetch (one point on every path through a row, before its stores)
    __device__ __forceinline__ void landed() {
        asm volatile("" ::"v"(dnext.x), "v"(dnext.y), "v"(dnext.z), "v"(dnext.w));
    }
    __device__ __forceinline__ void commit(int lane) {
        __builtin_amdgcn_wave_barrier();   // after every read of the current copy
        if (lane < dnc) dbuf[lane] = dnext;
        __builtin_amdgcn_wave_barrier();
    }

    // Entry `rel`.  The mask keeps even an inconsistent row inside the wave's slice.
    __device__ __forceinline__ void put(int32_t rel, int32_t col, float l) {
        stage[(uint32_t)rel & (uint32_t)STAGE_CAP] = make_uint2((uint32_t)col, __float_as_uint(l));
    }
    __device__ __forceinline__ void fold() {
        wacc += (TW)wepl;
        wepl = 0.f;
    }
    // Write the n staged entries and add their share of b.  Lanes take consecutive
    // entries (neighbouring voxels along the path share the cache lines of x), in groups
    // of 256 without branches inside a group: all LDS reads, then all gathers (an entry
    // past the row reads x[0], one cache line for all of them, and counts 0), then the
    // stores, so that each kind of access is in flight together.  With packed coordinates
    // (PACK) the column and the brick address are computed from them; an entry whose
    // coordinates lie outside the grid reads element 0 of the copy.
    template <bool WB, bool HALF, bool PACK>
    __device__ __forceinline__ void flush_t(int n, int lane) {
        constexpr int G = 4;   // chunks of 64 entries per group
        n = n < STAGE_CAP + 1 ? n : STAGE_CAP + 1;
        const int m = store ? (n < len ? n : len) : 0;   // entries stored
        const bool cst = chord > 0.f;
        __builtin_amdgcn_wave_barrier();
        // the wave's output phase runs at a raised issue priority, back to 0 once the row's
        // b is stored (emit_rows_wave): its loads and stores go out while the other waves
        // of the SIMD walk their rows (the 64-job batch: step 44.2 -> 43.6 ms, same outputs)
        __builtin_amdgcn_s_setprio(2);
        for (int g0 = 0; g0 < n; g0 += G * WAVE) {
            uint2 v[G];
            float xv[G];
            uint32_t col[G], xi[G];
#pragma unroll
            for (int u = 0; u < G; ++u) v[u] = stage[g0 + u * WAVE + lane];   // < 1024: in the slice
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int e = g0 + u * WAVE + lane;
                if (PACK) {
                    const uint32_t ix = v[u].x & ((1u << PACK_Y) - 1u);
                    const uint32_t iy = (v[u].x >> PACK_Y) & ((1u << (PACK_Z - PACK_Y)) - 1u);
                    const uint32_t iz = v[u].x >> PACK_Z;
                    // (24-bit operands: x < 1024, y, z < 2048, bricks per row <= 128)
                    col[u] = __umul24(gn[0], __umul24(gn[1], iz) + iy) + ix;
                    const uint32_t brick = __umul24(__umul24(iz, nby) + (iy >> 3), nbx) + (ix >> 3);
                    const bool in = e < n && ix < gn[0] && iy < gn[1] && iz < gn[2];
                    xi[u] = in ? (brick << 6) + ((iy & 7u) << 3) + (ix & 7u) : 0u;
                } else {
                    col[u] = v[u].x;
                    xi[u] = (e < n && v[u].x < nvox) ? v[u].x : 0u;
                }
            }
            if (WB) {
                const PCT_GLOBAL float *src = PACK ? xb : x;
#pragma unroll
                for (int u = 0; u < G; ++u) xv[u] = src[xi[u]];
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int e = g0 + u * WAVE + lane;
                if (e < m) {
                    // non-temporal: nothing here reads the output again, and x is kept in L2
                    const float sv = cst ? chord : __uint_as_float(v[u].y);
                    __builtin_nontemporal_store((int32_t)col[u], &cols[e]);
                    if (HALF) __builtin_nontemporal_store((uint16_t)__half_as_ushort(__float2half_rn(sv)), &vh[e]);
                    else __builtin_nontemporal_store(sv, &vf[e]);
                }
            }
            if (WB) {
#pragma unroll
                for (int u = 0; u < G; ++u) {
                    const int e = g0 + u * WAVE + lane;
                    wepl = fmaf(e < n ? __uint_as_float(v[u].y) : 0.f, xv[u], wepl);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
    }
    template <bool PACK>
    __device__ __forceinline__ void flush_p(int n, int lane) {
        if (want_b) {
            if (half) flush_t<true, true, PACK>(n, lane);
            else flush_t<true, false, PACK>(n, lane);
        } else {
            if (half) flush_t<false, true, PACK>(n, lane);
            else flush_t<false, false, PACK>(n, lane);
        }
    }
    // rows of a job with a bricked copy of x hold packed coordinates
    __device__ __forceinline__ void flush(int n, int lane) {
        if (pack) flush_p<true>(n, lane);
        else flush_p<false>(n, lane);
    }
};

// Entries closed inside a lane: the first one (`head`; it began in an earlier lane) is
// kept back for the stitch; `pend` is the open entry's length at the lane's end.
struct Walker {
    float head, pend;
    int done;
    int32_t cur;
};

// Item with at most one crossing per axis.  The displacement and the distance to the
// face are taken in R from the positions (no cancellation for an item nearly parallel to
// a face); their ratio -- the crossing's parameter in the item -- and the piece lengths
// are FP32.  The face distance F - (I + 1) or F - I equals the position in the voxel
// (F - I, exact) less 1 or 0, bit for bit.  The crossings are ordered by parameter, ties
// keeping the lower axis.  The item closes up to DIM entries, staged at the lane's next
// slots (Pc + done ...); a close with no crossing behind it writes the lane's next slot
// instead, which a later store of the wave overwrites in program order (this lane's next
// entry, the head of the next lane with a crossing, or the row's last entry), so every
// lane stores on every item without a branch.
template <typename R, int DIM, typename TW>
__device__ __forceinline__ void item_fast(const float hf[3], const int32_t stride[3], const int Ip[3],
                                          const R Fp[3], const int Ie[3], const R Fe[3], Walker &wk,
                                          RowOut<TW> &out, int Pc) {
    float lam[3] = {2.f, 2.f, 2.f}, dn2 = 0.f;
    int32_t dc[3] = {0, 0, 0};
    int tot = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int di = Ie[d] - Ip[d];   // -1, 0 or 1
        const float dff = (float)(Fe[d] - Fp[d]);
        const float dm = dff * hf[d];
        dn2 = fmaf(dm, dm, dn2);
        // distance to the face crossed, in R and rounded once: near a face its absolute
        // error must stay small, since a chord nearly parallel to the face divides it by a
        // small displacement
        const float dist = (float)(Fp[d] - R(Ip[d] + (di > 0 ? 1 : 0)));
        // in [0, 1] (a NaN from a vanishing displacement becomes 1: the item's end)
        lam[d] = di != 0 ? fminf(fabsf(dist) * __builtin_amdgcn_rcpf(fabsf(dff)), 1.f) : 2.f;
        dc[d] = di * stride[d];
        tot += di != 0 ? 1 : 0;
    }
    const float len = __builtin_amdgcn_sqrtf(dn2);
    // parameters in order, and the column steps of the first and the last crossing axis
    float l0, l1, l2 = 2.f;
    int32_t dfirst, dlast;
    if (DIM == 3) {
        const bool c10 = lam[1] < lam[0], c20 = lam[2] < lam[0], c21 = lam[2] < lam[1];
        l0 = fminf(fminf(lam[0], lam[1]), lam[2]);
        l1 = __builtin_amdgcn_fmed3f(lam[0], lam[1], lam[2]);
        l2 = fmaxf(fmaxf(lam[0], lam[1]), lam[2]);
        dfirst = (!c10 && !c20) ? dc[0] : ((c10 && !c21) ? dc[1] : dc[2]);
        dlast = (c10 && c20) ? dc[0] : ((!c10 && c21) ? dc[1] : dc[2]);
    } else {
        // (the parameters are never NaN: a select is the minimum and the maximum)
        const bool c10 = lam[1] < lam[0];
        l0 = c10 ? lam[1] : lam[0];
        l1 = c10 ? lam[0] : lam[1];
        dfirst = c10 ? dc[1] : dc[0];
        dlast = c10 ? dc[0] : dc[1];
    }
    const int32_t dsum = DIM == 3 ? dc[0] + dc[1] + dc[2] : dc[0] + dc[1];
    const int base = wk.done, slot = Pc + base;
    // first crossing: closes the entry open at the item's start
    const float len0 = fmaf(l0, len, wk.pend);
    wk.head = (base == 0 && tot > 0) ? len0 : wk.head;   // the lane's first entry
    out.put(slot, wk.cur, len0);
    const int32_t cur1 = wk.cur + dfirst;
    out.put(slot + (tot < 1 ? tot : 1), cur1, (l1 - l0) * len);   // second crossing
    if (DIM == 3)   // third crossing
        out.put(slot + (tot < 2 ? tot : 2), cur1 + dsum - dfirst - dlast, (l2 - l1) * len);
    const float lp = DIM == 3 && tot > 2 ? l2 : (tot > 1 ? l1 : (tot > 0 ? l0 : 0.f));
    wk.cur += dsum;
    wk.done = base + tot;
    wk.pend = (tot == 0 ? wk.pend : 0.f) + (1.f - lp) * len;
}

// Item of a straight row (one ray, every item crossing each axis at most once), measured
// in the ray's parameter t (the item runs from t_p to t_p + dt): the distance to a face
// over the axis' rate |c1| gives the crossing's offset in t, and the length of an offset
// is its product with Lt, the ray's length per unit of t.  The same crossings, in the
// same order, as item_fast; no per-item square root or reciprocal.
template <typename R, int DIM, class F>
__device__ __forceinline__ void item_ray(const float inv_rate[3], float Lt, float dt, const int32_t stride[3],
                                         const int Ip[3], const R frp[3], const int Ie[3], Walker &wk, F &&close) {
    float lam[3] = {3.f, 3.f, 3.f};
    int32_t dcol[3] = {0, 0, 0};
    int tot = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int di = Ie[d] - Ip[d];
        const bool up = di > 0;
        const float dist = (float)(frp[d] - (up ? R(1) : R(0)));   // minus the distance when up
        lam[d] = di != 0 ? fabsf(dist) * inv_rate[d] : 3.f;
        dcol[d] = up ? stride[d] : -stride[d];
        tot += di != 0 ? 1 : 0;
    }
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
        const float lc = fminf(fmaxf(lam[k], lp), dt);   // lam is never NaN
        close(k, go, wk.cur, k == 0 ? wk.pend + (lc - lp) * Lt : (lc - lp) * Lt);
        wk.cur += go ? dcol[k] : 0;
        lp = go ? lc : lp;
    }
    wk.pend = (tot == 0 ? wk.pend : 0.f) + (dt - lp) * Lt;
}

// Item with any number of crossings per axis (a chord longer than a voxel).  As in the
// fast form, distances to the faces are taken in R and the crossing parameters in FP32.
template <typename R, int DIM, class F>
__device__ __forceinline__ void item_general(const float hf[3], const int32_t stride[3], const int Ip[3],
                                             const R Fp[3], const R frp[3], const int Ie[3], const R Fe[3],
                                             Walker &wk, F &&close) {
    int bud[3] = {0, 0, 0}, st[3] = {1, 1, 1}, k[3] = {0, 0, 0}, tot = 0;
    float inv[3] = {0.f, 0.f, 0.f}, d0[3] = {0.f, 0.f, 0.f};
    float dn2 = 0.f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const int dd = Ie[d] - Ip[d];
        bud[d] = abs(dd);
        st[d] = dd > 0 ? 1 : -1;
        tot += bud[d];
        const float dff = (float)(Fe[d] - Fp[d]);
        inv[d] = __builtin_amdgcn_rcpf(fabsf(dff));
        d0[d] = fabsf((float)(frp[d] - (dd > 0 ? R(1) : R(0))));   // distance to the first face
        const float dm = dff * hf[d];
        dn2 = fmaf(dm, dm, dn2);
    }
    const float len = __builtin_amdgcn_sqrtf(dn2);
    float lp = 0.f;
    while (tot > 0) {
        int a = -1;
        float la = 0.f;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            if (bud[d] > 0) {
                const float ld = (d0[d] + (float)k[d]) * inv[d];
                if (a < 0 || ld < la) {
                    a = d;
                    la = ld;
                }
            }
        }
        float lc = la > lp ? la : lp;
        lc = lc < 1.f ? lc : 1.f;
        close(-1, true, wk.cur, wk.pend + (lc - lp) * len);
        wk.pend = 0.f;
        lp = lc;
#pragma unroll
        for (int d = 0; d < DIM; ++d)
            if (d == a) {
                wk.cur += st[d] * stride[d];
                bud[d] -= 1;
                k[d] += 1;
            }
        --tot;
    }
    wk.pend += (1.f - lp) * len;
}

// ------------------------------------------------------------------ the row walk
template <int DIM>
__device__ __forceinline__ int32_t col_at(const int32_t stride[3], const int I[3]) {
    return DIM == 3 ? I[0] + stride[1] * I[1] + stride[2] * I[2] : I[0] + stride[1] * I[1];
}

// What a staged entry holds for its voxel: the column, or for a job with a bricked copy
// of x its packed coordinates (x in bits 0-9, y in bits 10-20, z in bits 21-31),
// which the copy-out turns into the column and the brick address.  Both are sums of the
// per-axis steps below, so the walks that stage entries use them unchanged.
template <int DIM>
__device__ __forceinline__ void stage_strides(const JobDev &J, int32_t stride[3]) {
    const bool pack = J.xb != nullptr;
    stride[0] = 1;
    stride[1] = pack ? (1 << PACK_Y) : J.n[0];
    stride[2] = pack ? (1 << PACK_Z) : J.n[0] * J.n[1];
}

// Walk one row with the whole wave; n_entries = entries produced.
// FAST: every item crosses each axis at most once (the row's `fast` flag).
// RAY: a straight row (kind 1) with FAST: every lane takes the one ray, whose constants
// are the same in all lanes.
template <typename R, int DIM, typename TW, bool FAST, bool RAY = false>
__device__ __forceinline__ void wave_row(const JobDev &J, LdsRow wl, int kind, RowOut<TW> &out,
                                         int lane, int64_t &n_entries) {
    // item counts as the count pass writes them; the bounds only matter for a
    // description it did not write (the walk then stays finite and the count check fails)
    const int mmax = J.nmax + 1;
    const int M0 = min(max(RL_I32(wl, ray[0].M), 0), mmax);
    const int Ns = (!RAY && kind == 2) ? min(max(RL_I32(wl, spl.N), 0), (1 << 22) + 1) : 0;
    const int M1 = (!RAY && kind == 2) ? min(max(RL_I32(wl, ray[1].M), 0), mmax) : 0;
    const int T = M0 + Ns + M1;
    n_entries = 0;
    if (T == 0) return;
    // items per lane: the smallest K with which the three lane groups fit the wave
    int K = (T + WAVE - 1) / WAVE, L0, Ls, L1;
    for (;;) {
        L0 = (M0 + K - 1) / K;
        Ls = (Ns + K - 1) / K;
        L1 = (M1 + K - 1) / K;
        if (L0 + Ls + L1 <= WAVE) break;
        ++K;
    }
    const int last_lane = L0 + Ls + L1 - 1;
    LaneP<R> P;
    int base = 0;
    const bool spl = !RAY && lane >= L0 && lane < L0 + Ls;
    // each lane its piece, from the wave's LDS copy of the description (the lanes of a
    // curved row read different pieces)
    if (RAY || lane < L0) {
        lane_ray<R, DIM, 0>(J, wl, P);
        base = lane * K;
    } else if (spl) {
        lane_spline<R, DIM>(J, wl, P);
        base = (lane - L0) * K;
    } else {
        lane_ray<R, DIM, 1>(J, wl, P);
        base = (lane - L0 - Ls) * K;
    }
    P.M = RAY ? M0 : ((lane < L0) ? M0 : (spl ? Ns : (lane <= last_lane ? M1 : 0)));
    // items [first, last); a lane past the pieces has the empty range at 0
    const bool has_items = base < P.M;
    const int first = has_items ? base : 0;
    const int last = has_items ? ((base + K < P.M) ? base + K : P.M) : 0;
    if (!has_items) {
        P.tS = R(0);
        P.tE = R(0);
    }
    int32_t stride[3];
    stage_strides<DIM>(J, stride);
    const float hf[3] = {(float)J.h[0], (float)J.h[1], (float)J.h[2]};

    // pass 1: voxel at the first item end, crossings up to the last one.  Per axis, the
    // difference of the end indices, or, where the lane's items reach into one of the
    // axis' turning windows (the coordinate need not be monotone there), the sum of that
    // axis' index steps over the lane's items -- the same count, axis by axis, that a walk
    // of all the items' voxels would give.  Only the axes some lane must walk are walked.
    int Is[3] = {0, 0, 0};
    R Fs[3] = {R(0), R(0), R(0)}, frs[3] = {R(0), R(0), R(0)};
    int c = 0;
    {
        piece_point<R, DIM>(P, first, R(first), Fs);
        piece_voxel<R, DIM>(P, Fs, Is, frs);
        R Fe[3], fre[3];
        int Ie[3];
        piece_point<R, DIM>(P, last, R(last), Fe);
        piece_voxel<R, DIM>(P, Fe, Ie, fre);
        bool walk[3] = {false, false, false};
        if (spl) {
            // the turning windows from the LDS copy, all read before any is used
            int32_t win[3][4];
#pragma unroll
            for (int d = 0; d < DIM; ++d)
#pragma unroll
                for (int k = 0; k < 4; ++k) win[d][k] = RV(wl, spl.win[d][k]);
#pragma unroll
            for (int d = 0; d < DIM; ++d)
                walk[d] = ((first < win[d][1]) & (last > win[d][0])) | ((first < win[d][3]) & (last > win[d][2]));
        }
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            int cd = abs(Ie[d] - Is[d]);
            if (__builtin_amdgcn_ballot_w64(walk[d]) != 0) {   // uniform
                int steps = 0, Ip = Is[d];
                for (int it = 0; it < K; ++it) {
                    const int m = min(first + it + 1, last);   // item end (the last one again past it)
                    const int I = axis_index<R>(P, d, R(m));
                    steps += abs(I - Ip);
                    Ip = I;
                }
                cd = walk[d] ? steps : cd;
            }
            c += cd;
        }
    }
    int ctot;
    const int Pc = wave_excl_scan(c, ctot);

    // pass 2: the pieces of every item
    Walker wk;
    wk.head = 0.f;
    wk.pend = 0.f;
    wk.done = 0;
    wk.cur = col_at<DIM>(stride, Is);
    const int32_t col_start = wk.cur;
    // every lane stores on every call, without a branch: a lane without an entry here
    // writes the slot of its next entry, which a later store of the wave (this lane's
    // next entry, the head of the next lane with a crossing, or the row's last entry)
    // overwrites in program order
    auto close = [&](int k, bool ok, int32_t col, float len) {
        (void)k;
        wk.head = (ok && wk.done == 0) ? len : wk.head;
        out.put(Pc + wk.done, col, len);
        wk.done += ok ? 1 : 0;
    };
    {
        int Ip[3] = {Is[0], Is[1], Is[2]};
        R Fp[3] = {Fs[0], Fs[1], Fs[2]}, frp[3] = {frs[0], frs[1], frs[2]};
        // every lane runs K items: past its last item end it takes that end again, an
        // empty item (the same point, bit for bit: no crossing, no length), so the loop
        // has no branch
        // the ray's constants (straight rows): rate of every axis per unit of t and the
        // length per unit of t
        float inv_rate[3] = {0.f, 0.f, 0.f}, Lt = 0.f;
        R tp = r_fmin<R>(r_fmax<R>(R(first), P.tS), P.tE);
        if (RAY) {
            float l2 = 0.f;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const float r = fabsf((float)P.c1[d]);
                inv_rate[d] = 1.f / r;
                const float q = r * hf[d];
                l2 = fmaf(q, q, l2);
            }
            Lt = sqrtf(l2);
        }
#pragma unroll 2
        for (int it = 0; it < K; ++it) {
            const int m = min(first + it + 1, last);   // item end
            const R mf = R(m);
            R Fe[3], fre[3];
            int Ie[3];
            if (RAY) {
                // linear item ends: F(t) = c0 + c1 t
                const R t = r_fmin<R>(mf, P.tE);
#pragma unroll
                for (int d = 0; d < 3; ++d) Fe[d] = d < DIM ? r_fma<R>(P.c1[d], t, P.c0[d]) : R(0);
                piece_voxel<R, DIM>(P, Fe, Ie, fre);
                item_ray<R, DIM>(inv_rate, Lt, (float)(t - tp), stride, Ip, frp, Ie, wk, close);
                tp = t;
            } else {
                piece_next<R, DIM>(P, m, mf, Fe);
                piece_voxel<R, DIM>(P, Fe, Ie, fre);
                if (FAST) item_fast<R, DIM>(hf, stride, Ip, Fp, Ie, Fe, wk, out, Pc);
                else item_general<R, DIM>(hf, stride, Ip, Fp, frp, Ie, Fe, wk, close);
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                Ip[d] = Ie[d];
                Fp[d] = Fe[d];
                frp[d] = fre[d];
            }
        }
        // a lane past the pieces walked a point that need not exist: nothing of it is kept
        if (!has_items) wk.pend = 0.f;
    }

    // every lane must have closed exactly the crossings it counted in pass 1
    const bool lane_ok = wk.done == c;

    // stitch: the entry open at a lane's start gets the tail of the last lane with a
    // crossing before it, the whole lengths of the lanes in between, and this lane's head
    const bool f = c > 0;
    int fs = f ? 1 : 0;
    float vs = wk.pend;
    wave_seg_scan(vs, fs);
    float Oin = lane_prev(vs);   // open length before this lane
    if (lane == 0) Oin = 0.f;
    if (f) out.put(Pc, col_start, Oin + wk.head);
    const float Oend = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, vs), last_lane));
    const int32_t ocol = __builtin_amdgcn_readlane(wk.cur, last_lane);
    if (lane == 0) out.put(ctot, ocol, Oend);
    out.bad |= !lane_ok;
    n_entries = (int64_t)ctot + 1;   // staged; the caller writes them out
}

// Straight row (kind 1) in the mixed form, by crossings instead of items.  The lanes
// split the items as in wave_row and count their crossings the same way (index
// differences at the ends of their stretches), so each lane owns the same crossings.
// A lane then takes them in the order of the ray parameter t: along axis d they lie at
// tA_d + k / |c1_d|, k = 0 .. n_d - 1 (tA_d: the first face ahead of the stretch's
// start), and the next one is the smallest parameter among the axes with crossings
// left (ties keep the lower axis).  The entry closed there is as long as the step in t
// since the row's previous crossing times the length per unit of t.  For a lane's first
// entry that previous crossing is the nearest face behind the stretch's start (or the
// row's start point), so no lane needs the others' lengths and there is nothing to
// stitch.  Parameters are FP64; a parameter step is rounded to FP32 once.
template <int DIM, typename TW>
__device__ __forceinline__ void wave_ray_row(const JobDev &J, RowRefD<double, DIM> w, LdsRow wl, RowOut<TW> &out,
                                             int lane, int64_t &n_entries) {
    using R = double;
    const int M = min(max(RL_I32(wl, ray[0].M), 0), J.nmax + 1);
    n_entries = 0;
    if (M == 0) return;
    const int K = (M + WAVE - 1) / WAVE;
    const int last_lane = (M + K - 1) / K - 1;
    LaneP<R> P;
    // the ray, the same in every lane, with scalar loads (read from the LDS copy it was
    // as fast in 2D and 1% slower in 3D)
    lane_ray<R, DIM, 0>(J, w, P);
    const int base = lane * K;
    const bool has_items = base < M;
    const int first = has_items ? base : 0;
    const int last = has_items ? min(base + K, M) : 0;
    if (!has_items) {
        P.tS = R(0);
        P.tE = R(0);
    }
    // the stretch's ends (item ends first and last) and its crossings per axis
    R Fs[3], frs[3], Fe[3], fre[3];
    int Is[3], Ie[3];
    piece_point<R, DIM>(P, first, R(first), Fs);
    piece_voxel<R, DIM>(P, Fs, Is, frs);
    piece_point<R, DIM>(P, last, R(last), Fe);
    piece_voxel<R, DIM>(P, Fe, Ie, fre);
    const R ta = r_fmin<R>(r_fmax<R>(R(first), P.tS), P.tE);
    const R tb = r_fmin<R>(r_fmax<R>(R(last), P.tS), P.tE);
    int n[3] = {0, 0, 0};
    int c = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        n[d] = abs(Ie[d] - Is[d]);
        c += n[d];
    }
    int ctot;
    const int Pc = wave_excl_scan(c, ctot);

    int32_t stride[3];
    stage_strides<DIM>(J, stride);
    R inv[3] = {R(0), R(0), R(0)}, tA[3] = {R(0), R(0), R(0)};
    int32_t dcol[3] = {0, 0, 0};
    R tprev = P.tS;   // the row's start point, unless a face lies between it and ta
    float l2 = 0.f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R rate = fabs(P.c1[d]);   // voxels per unit of t; 1 on the dominant axis
        const float q = (float)rate * (float)J.h[d];
        l2 = fmaf(q, q, l2);
        // 1 / rate: the hardware reciprocal and one Newton step (unused when rate = 0)
        R iv = __builtin_amdgcn_rcp(rate);
        iv = r_fma<R>(r_fma<R>(-rate, iv, R(1)), iv, iv);
        inv[d] = iv;
        const bool up = P.c1[d] > R(0);
        // distance from the start to the first face ahead and to the nearest face behind
        const R ahead = up ? R(1) - frs[d] : frs[d];
        const R behind = up ? frs[d] : R(1) - frs[d];
        tA[d] = r_fma<R>(ahead, iv, ta);
        if (rate > R(0)) tprev = r_fmax<R>(tprev, r_fma<R>(-behind, iv, ta));
        dcol[d] = up ? stride[d] : -stride[d];
    }
    tprev = r_fmin<R>(tprev, ta);
    const float Lt = sqrtf(l2);   // mm per unit of t

    int32_t cur = col_at<DIM>(stride, Is);
    int k0 = 0, k1 = 0, k2 = 0;
    R tn0 = tA[0], tn1 = tA[1], tn2 = tA[2];
    for (int j = 0; j < c; ++j) {
        const bool v0 = k0 < n[0], v1 = k1 < n[1];
        const bool a1 = v1 && (!v0 || tn1 < tn0);
        R tc = a1 ? tn1 : tn0;
        int32_t dc = a1 ? dcol[1] : dcol[0];
        bool a2 = false;
        if (DIM == 3) {
            a2 = (k2 < n[2]) && (!(v0 || v1) || tn2 < tc);
            tc = a2 ? tn2 : tc;
            dc = a2 ? dcol[2] : dc;
        }
        // tc >= tprev: each axis' parameters grow with k (an fma with a positive
        // reciprocal rounds monotonically), the smallest of them never falls below the
        // last one taken, and the first is at or past ta, which bounds tprev
        out.put(Pc + j, cur, (float)(tc - tprev) * Lt);
        cur += dc;
        tprev = tc;
        k0 += (!a1 && !a2) ? 1 : 0;
        k1 += (a1 && !a2) ? 1 : 0;
        tn0 = r_fma<R>(R(k0), inv[0], tA[0]);
        tn1 = r_fma<R>(R(k1), inv[1], tA[1]);
        if (DIM == 3) {
            k2 += a2 ? 1 : 0;
            tn2 = r_fma<R>(R(k2), inv[2], tA[2]);
        }
    }
    // the row's last entry: from its last crossing to the end point
    if (lane == last_lane) out.put(ctot, cur, (float)r_fmax<R>(tb - tprev, R(0)) * Lt);
    n_entries = (int64_t)ctot + 1;   // staged; the caller writes them out
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

// Largest |F'(m)| = |c1 + 2 c2 m + 3 c3 m^2| over [0, N]: at an end or at the vertex.
template <typename R>
__device__ __forceinline__ R spline_max_rate(R c1, R c2, R c3, int N) {
    const R qa = R(3) * c3, qb = R(2) * c2, n = R(N);
    const R g0 = c1;
    const R g1 = r_fma<R>(r_fma<R>(qa, n, qb), n, c1);
    R g = r_fmax<R>(g0 < R(0) ? -g0 : g0, g1 < R(0) ? -g1 : g1);
    if (qa != R(0)) {
        const R mv = -qb / (R(2) * qa);
        if (mv > R(0) && mv < n) {
            const R gv = r_fma<R>(r_fma<R>(qa, mv, qb), mv, c1);
            g = r_fmax<R>(g, gv < R(0) ? -gv : gv);
        }
    }
    return g;
}

// What the count pass learns while it describes a row: its kind and, for kinds 1 and 2,
// its number of CSR entries (1 + the face crossings of its pieces, counted from the
// pieces as they are written, with the arithmetic the emit applies to them).
struct RowSetup {
    int kind;
    int64_t n;
};

template <typename R, int DIM>
__device__ __forceinline__ RowSetup setup_row(const JobDev &J, int64_t g, RowRefD<R, DIM> w) {
    PathGeom<R> p;
    if (J.path == 1) make_path<R, DIM, true>(J, g, p);
    else make_path<R, DIM, false>(J, g, p);
    const R ninf = -r_inf<R>(), pinf = r_inf<R>();
    int kind = 0, fast = 1;   // fast: every item crosses each axis at most once
    int64_t cross = 0;        // face crossings of the pieces
    bool any = false;         // a piece with items
    RV(w, spl.N) = 0;
    RV(w, ray[1].M) = 0;
    if (!p.curved) {
        R lo = ninf, hi = pinf;
        const bool hit = clip_box<R, DIM>(J, p.Q, p.u, lo, hi);
        kind = hit ? 1 : 0;
        LaneP<R> lp;
        if (!make_ray<R, DIM, 0>(J, p.Q, p.u, lo, hi, hit, w, lp)) fast = 0;
        if (lp.M > 0) {
            cross += ray_piece_crossings<R, DIM>(lp);
            any = true;
        }
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
        kind = in ? 2 : 3;
        RV(w, ray[0].M) = 0;
        if (in) {
            R lo = ninf, hi = R(0);
            bool hit = clip_box<R, DIM>(J, p.P0, p.d0, lo, hi);
            LaneP<R> lp;
            if (!make_ray<R, DIM, 0>(J, p.P0, p.d0, lo, hi, hit, w, lp)) fast = 0;
            if (lp.M > 0) cross += ray_piece_crossings<R, DIM>(lp);
            lo = R(0);
            hi = pinf;
            hit = clip_box<R, DIM>(J, p.P1, p.d1, lo, hi);
            if (!make_ray<R, DIM, 1>(J, p.P1, p.d1, lo, hi, hit, w, lp)) fast = 0;
            if (lp.M > 0) cross += ray_piece_crossings<R, DIM>(lp);
            any = true;   // the spline has N >= 1 items
            // the spline as the emit reads it back (lane_spline): t in [0, N], the grid's range
            LaneP<R> sp;
            sp.tS = R(0);
            sp.tE = R(p.N);
            sp.M = p.N;
            const R iN = p.invN, iN2 = iN * iN, iN3 = iN2 * iN;
            const R thr = sizeof(R) == 8 ? R(1e-9) : R(1e-2);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const R ih = (d < DIM) ? R(J.invh[d]) : R(0);
                const R fS = (d < DIM) ? (p.P0[d] - R(J.o[d])) * ih : R(0);
                const R c1 = p.c1[d] * ih * iN, c2 = p.c2[d] * ih * iN2, c3 = p.c3[d] * ih * iN3;
                RV(w, spl.c0[d]) = fS;
                RV(w, spl.c1[d]) = c1;
                RV(w, spl.c2[d]) = c2;
                RV(w, spl.c3[d]) = c3;
                int32_t win[4] = {-1, -1, -1, -1};
                if (d < DIM) {
                    spline_windows<R>(c1, c2, c3, p.N, thr, win);
                    // a chord moves less than one voxel along d when |F'| < 1 over [0, N]
                    if (!(spline_max_rate<R>(c1, c2, c3, p.N) < R(0.999))) fast = 0;
                    sp.c0[d] = fS;
                    sp.c1[d] = c1;
                    sp.c2[d] = c2;
                    sp.c3[d] = c3;
                    sp.lo[d] = 0;
                    sp.hi[d] = J.n[d] - 1;
                    cross += spline_axis_crossings<R>(sp, d, win);
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) RV(w, spl.win[d][k]) = win[k];
            }
            RV(w, spl.N) = p.N;
        }
    }
    RV(w, kind) = kind;
    RV(w, fast) = fast;
    double bfac = 1.0;
    if (J.noise > 0.0) {
        R z1, z2;
        normal_pair<R>(J.seed, 4, (uint64_t)g, z1, z2);
        bfac = (double)(R(1) + R(J.noise) * z1);
    }
    RV(w, bfac) = bfac;
    return RowSetup{kind, (kind == 1 || kind == 2) && any ? cross + 1 : 0};
}

// Number of CSR entries of a row described by w (one lane): for kinds 1 and 2 the count
// setup_row took (1 + the face crossings of its items, exactly as wave_row produces
// them); the per-lane walk for kind 3.  A row with more entries than a wave stages
// becomes kind 3 here (lane_walk: the row is the per-lane kernel's).
template <typename R, int DIM>
__device__ __forceinline__ int64_t count_row(const JobDev &J, RowRefD<R, DIM> w, int64_t g, const RowSetup &su,
                                             int &lane_walk) {
    lane_walk = su.kind == 3 ? 1 : 0;
    if (su.kind == 0) return 0;
    if (su.kind == 3) {
        CountSink s;
        trace_row<R, DIM, true>(J, g, s);
        return s.n;
    }
    const int64_t n = su.n;
    if (n > STAGE_CAP) {
        lane_walk = 1;
        // more entries than the wave's LDS slice holds: the per-lane walk takes the row
        RV(w, kind) = 3;
        CountSink s;
        trace_row<R, DIM, true>(J, g, s);
        return s.n;
    }
    return n;
}

// Emit pass over rows [r0, r0 + nr) of job J by one wavefront.  stage: the wave's LDS
// slice; its last STAGE_DESC slots hold the copy of the current row's description.
template <typename R, int DIM, bool STORE>
__device__ __forceinline__ void emit_rows_wave(const JobDev &J, char *rowbuf, int64_t r0, int nr, int lane,
                                               uint2 *stage, int32_t *status) {
    using TW = typename std::conditional<std::is_same<R, double>::value, double, float>::type;
    constexpr int NC = (int)(rv_bytes<R>() / 16);
    static_assert(NC <= WAVE && 2 * NC <= STAGE_DESC, "a description is copied with one chunk per lane");
    uint4 *dbuf = reinterpret_cast<uint4 *>(stage + STAGE_ROW_MAX);
    const int64_t rend = (r0 + nr < J.row_count) ? r0 + nr : J.row_count;
    if (r0 < rend && lane < NC) dbuf[lane] = row_ref<R, DIM>(rowbuf, J, r0).template at<uint4>((size_t)lane * 16);
    __builtin_amdgcn_wave_barrier();
    const LdsRow wl{(char *)dbuf};
    // the rows' CSR bounds, read once per wave (lane l: row_ptr[r0 + l] and the next), so
    // that a row takes its pair with readlane instead of a trip to memory
    int64_t rp_a = 0, rp_b = 0;
    if (STORE && r0 + lane < rend) {
        rp_a = J.row_ptr[r0 + lane];
        rp_b = J.row_ptr[r0 + lane + 1];
    }
    // waited for here, once: a use inside the row loop would make every row wait for all
    // of its loads and stores in flight
    asm volatile("" ::"v"(rp_a), "v"(rp_b));
    bool bad = false;
    for (int64_t r = r0; r < rend; ++r) {
        RowOut<TW> out;
        out.dbuf = dbuf;
        out.dnc = NC;
        out.dnext = make_uint4(0u, 0u, 0u, 0u);
        if (lane < NC)   // the next row's description (the last row's own at the end of the range)
            out.dnext = row_ref<R, DIM>(rowbuf, J, r + 1 < rend ? r + 1 : r).template at<uint4>((size_t)lane * 16);
        // (the control fields from the LDS copy, which holds this row's description)
        const int kind = RL_I32(wl, kind);
        const int fast = RL_I32(wl, fast);
        const double bfac = RL_F64(wl, bfac);
        const bool valid = kind >= 0 && kind <= 3;
        if (!valid && lane == 0) set_status_dev(status, PCT_EINTERNAL);   // not a description of the count pass
        const bool mine = valid && kind != 3;   // kind 3: walked by the per-lane kernel
        out.x = gptr(J.x);
        out.pack = J.xb != nullptr;
        out.xb = gptr((const float *)J.xb);
        out.gn[0] = (uint32_t)J.n[0];
        out.gn[1] = (uint32_t)J.n[1];
        out.gn[2] = (uint32_t)J.n[2];
        out.nbx = (uint32_t)J.nbx;
        out.nby = (uint32_t)J.nby;
        out.wepl = 0.f;
        out.wacc = TW(0);
        out.half = (J.val_dtype == PCT_F16);
        out.want_b = (J.b != nullptr);
        out.store = STORE && mine;
        out.bad = false;
        out.stage = stage;
        out.nvox = (uint32_t)J.n[0] * (uint32_t)J.n[1] * (uint32_t)(DIM == 3 ? J.n[2] : 1);
        out.len = 0;
        out.chord = J.chord;
        int64_t pos = 0;
        if (out.store) {
            const int i = (int)(r - r0);   // < 64
            pos = readlane_i64(rp_a, i);
            const int64_t end = readlane_i64(rp_b, i);
            if (pos < 0 || end < pos || end > J.cap) {
                if (lane == 0) set_status_dev(status, PCT_ECAPACITY);
                out.store = false;
                pos = 0;
            } else {
                out.len = (int32_t)(end - pos);
            }
        }
        out.cols = gptr(J.cols + pos);
        out.vh = gptr((uint16_t *)J.vals + pos);
        out.vf = gptr((float *)J.vals + pos);
        int64_t ne = 0;
        if (mine && kind != 0) {
            if constexpr (std::is_same<R, double>::value) {
                if (kind == 1) wave_ray_row<DIM, TW>(J, row_ref<R, DIM>(rowbuf, J, r), wl, out, lane, ne);
                else if (fast) wave_row<R, DIM, TW, true>(J, wl, kind, out, lane, ne);
                else wave_row<R, DIM, TW, false>(J, wl, kind, out, lane, ne);
            } else {
                if (fast) {
                    if (kind == 1) wave_row<R, DIM, TW, true, true>(J, wl, kind, out, lane, ne);
                    else wave_row<R, DIM, TW, true>(J, wl, kind, out, lane, ne);
                } else {
                    wave_row<R, DIM, TW, false>(J, wl, kind, out, lane, ne);
                }
            }
        }
        // the next row's description: before the row's stores and gathers, unless the
        // row's entries reach into the slots of the copy
        out.landed();
        if (ne <= STAGE_ROW_MAX) {
            out.commit(lane);
            if (ne > 0) {
                out.flush((int)ne, lane);
                out.fold();
            }
        } else {
            out.flush((int)min(ne, (int64_t)(STAGE_CAP + 1)), lane);
            out.fold();
            out.commit(lane);
        }
        if (mine) {
            bad |= out.bad;
            if (STORE && out.store && ne != out.len && lane == 0) set_status_dev(status, PCT_EINTERNAL);
            if (out.want_b) {
                const TW bs = (TW)wave_sum((double)out.wacc);
                if (lane == 0) *gptr(J.b + r) = (float)(bs * (TW)bfac);
            }
        }
        __builtin_amdgcn_s_setprio(0);   // raised by the row's flush
    }
    if (__builtin_amdgcn_ballot_w64(bad) != 0 && lane == 0) set_status_dev(status, PCT_EINTERNAL);
}

// Rows whose spline may leave the box (kind 3): one lane per row, general walk.
template <typename R, int DIM, bool STORE>
__device__ __forceinline__ void emit_row_lane(const JobDev &J, RowRefD<R, DIM> w, int64_t r, int32_t *status) {
    using TW = typename std::conditional<std::is_same<R, double>::value, double, float>::type;
    EmitSink<R, TW> s;
    s.cols = J.cols;
    s.vals = J.vals;
    s.x = J.x;
    s.half = (J.val_dtype == PCT_F16);
    s.want_b = (J.b != nullptr);
    s.store = STORE;
    s.chord = J.chord;
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
    if (s.want_b) J.b[r] = (float)(s.wepl * (TW)RV(w, bfac));
}

}  // namespace pct
